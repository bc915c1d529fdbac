// kernel.h -- the NGDBF decode kernel for gfx950 (device code), shared by
// the translation units that instantiate its variants.
//
// Data layout.
//   HBM: y frame-major [F][n] (float32 or int8), sigma [F], outputs
//        out_bits [F][ceil(n/8)], out_iters [F], out_converged [F].
//   Code tables: uint16 N(i) (CSR) and M(k) (CSC), staged into LDS once per
//        workgroup (read from global memory by the base kernel with two or
//        more waves per frame).
//   LDS per frame: syndrome bits s, per-bit counts u_k of unsatisfied checks,
//        the unsatisfied-check count, an x / flip bit row, a toggle row and a
//        toggle-event list; the base kernel's flip counts; for the extended
//        decoders also two reduction words and, with noise reuse, the frame's
//        sample stream.  Per wavefront a small Box-Muller work list.
//   Registers: each lane owns QPL bit quads (bits 4j .. 4j+3) and keeps their
//        saturated y_k, smoothing counters and decisions (the extended
//        decoders also their thresholds theta_k; the base decoder keeps a
//        table of theta lambda^u in LDS and per-bit flip counts instead).
//
// Frames are independent (Sec. IV): one wavefront decodes a frame of up to
// 1024 bits with no workgroup barrier in its round loop; longer codes use
// several wavefronts per frame.  Every round runs on chip; HBM sees y once
// and the decoded bits once per frame.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

#include "../../include/ngdbf.h"
#include "noise.h"

namespace ngdbf {

constexpr int kWave = 64;
// Box-Muller work-list entries per wavefront (pairs whose flip decision the
// radius bound could not settle); past this a lane transforms its own pairs.
constexpr int kListCap = 256;
// a list entry: the pair's two Philox words, a_k and theta_k of both bits
constexpr int kEntryWords = 6;
// the base decoder's list: the pair's two Philox words, a_k of both bits and
// a tag (the pair's first bit k0 in bits 0-15, its owner lane in bits 16-21,
// the pair's slot 2r + p in that lane in bits 22-24; its thresholds are looked
// up when the list is finished); after the entries, one decision word per
// lane of the wave, into which the list's decisions are or-ed
constexpr int kListCapLazy = 192;
constexpr int kEntryWordsLazy = 5;
constexpr int kDecisionWords = 64;
// smoothing counters are 16-bit halves biased by this value
constexpr uint32_t kXBias = 32768u;
// s_setprio levels of the round phases of the base kernel and of the packed
// quantized decoder (which has no list): the later a phase is in the round,
// the higher it runs, so that the SIMD finishes the rounds it has started
// before it starts others (a frame of several waves meets its other waves at
// workgroup barriers; a wave that lags behind them catches up first).
constexpr int kPrioHead = 0, kPrioDense = 1, kPrioList = 2, kPrioSyndrome = 3;
constexpr int kPrioPackedHead = 1, kPrioPackedDense = 2, kPrioPackedSyndrome = 3;

// decode_kernel's EXT argument: which decoder family the instance holds
constexpr int kExtNone = 0;    // multi-bit, binary32, per-bit draws
constexpr int kExtMulti = 1;   // multi-bit with quantization and/or noise reuse
constexpr int kExtSingle = 2;  // single-bit flips (Step 3a)
constexpr int kExtSwitch = 3;  // mode switching (Step 3b, then 3a)
constexpr int kExtQuantReuse = 4;  // multi-bit, quantized, noise reuse: packed 16-bit lanes

// packed pairs of signed 16-bit integers (two bits of a quad per register)
typedef short short2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ short2_t as_s2(uint32_t v) { return __builtin_bit_cast(short2_t, v); }
__device__ __forceinline__ uint32_t as_u32(short2_t v) { return __builtin_bit_cast(uint32_t, v); }

// x_k g(y_k) of a bit that can never flip (past the code, or a NaN sample):
// with |g(w) S_k| <= 255 * 15 and |g(q_k)|, |theta~| <= 255, E~_k stays far
// above every threshold and within int16
constexpr int kNeverFlip = 16383;

struct DecodeArgs {
  // code tables, uint16, staged into LDS: col_idx (N(i), CSR) | row_idx
  // (M(k), CSC) | row_ptr | col_ptr (the pointers only for irregular codes)
  const uint32_t *tables;
  int32_t table_words;
  int32_t off_row, off_rowptr, off_colptr;  // uint16 offsets
  int32_t dv, dc;                           // uniform degrees, 0 if irregular
  int32_t n, m;
  const void *y;
  int64_t n_frames;
  const float *sigma;
  float sigma_scalar;
  float w, theta, lambda, eta, ymax;
  int32_t t_max, smooth_window;
  uint32_t key0, key1;
  uint64_t frame_base;
  uint8_t *out_bits;
  int32_t *out_iters;
  uint8_t *out_conv;
  uint8_t *trace;
  // segment mode (n_segments > 0): frame f of the launch belongs to the
  // segment s with offset_s <= f < offset_{s+1}; its data live at pool slot
  // first_slot_s + (f - offset_s) and its noise key is (seed_s,
  // frame_base_s + f - offset_s)
  const ngdbf_segment *segments;
  int32_t n_segments;
  int64_t pool_frames;                    // slots in the pools (segment mode)
  int32_t frames_per_block;               // frame slots per workgroup
  int32_t sw_words, uw_words, xw_words;   // per-slot LDS arrays
  uint32_t dc_recip;                      // ceil(2^20 / d_c) for regular codes
  int32_t event_cap;                      // check-toggle events per frame and round held
  uint32_t list_unsat_max;                // rounds starting with more unsatisfied checks
                                          // apply events without listing them
                                          // for the parallel u update (0: irregular code)
  int32_t slot_words;                     // LDS words per frame slot (even)
  int32_t slots_off;                      // LDS word offset of the frame slots (even)
  // extended decoders (EXT kernels)
  int32_t variant;      // 0 multi-bit (Step 3b), 1 single-bit (Step 3a), 2 mode switching
  int32_t quant_bits;   // 0: binary32; Q > 0: the Q-bit quantized decoder (Sec. IV-E)
  int32_t noise_reuse;  // 1: shift-register noise chain (Sec. V-B)
  float qc, qtop;       // quantizer scale fl32(N_Q / 2Y_max) and top level N_Q/2 - 1
  float wq;             // g(w) in half steps
  float qbound;         // N_Q - 1, the largest |g(q)| in half steps
  int32_t red_off;      // slot word offset of the two 64-bit reduction words (even)
  int32_t stream_off;   // slot word offset of the frame's sample stream
  int32_t stream_len;   // n + T - 1 samples per frame with noise reuse
  int32_t stream_q;     // ceil(stream_len / 4): sample i sits at (i & 3) * stream_q + (i >> 2)
  int32_t list_words;   // Box-Muller list words per wave (0 when no list is used)
  int32_t clear_words;  // slot words cleared per frame (the stream is rewritten)
  int32_t qtab_off;     // kExtQuantReuse: LDS word offset of theta~(u), u = 0..T (int16)
  int32_t stream_lr;    // kExtQuantReuse: int16 samples in the stream's row (a multiple of 4)
  // base decoder (kExtNone): theta lambda^u for u = 0..T (float, LDS word
  // offset) and the per-frame flip counts (two 16-bit counts per word: bits
  // 2i and 2i + 1; slot word offset)
  int32_t thr_off;
  int32_t fc_off;
  int32_t fc_bytes;     // 1: one 8-bit count per bit (T <= 255), 0: 16-bit counts
  uint64_t *stats;      // base kernel: [pairs evaluated, pairs transformed], or null
  // this launch's frame queue: kQueueLanes counters of handed-out runs (one
  // 128-byte line each) and the count of finished takers, zero at the start;
  // the last taker to finish sets them back to zero
  unsigned long long *queue;
  int32_t queue_chunk;  // consecutive frames per run (>= 1)
};

// A frame queue's counters: taker t draws from counter t % kQueueLanes, whose
// runs cover frames c + kQueueLanes * (chunk * i + 0 .. chunk - 1), so that no
// single counter carries every update.  Words between counters pad them to
// separate cache lines.
constexpr int kQueueLanes = 8;
constexpr int kQueueStride = 16;  // uint64 words per counter (128 bytes)
constexpr int kQueueWords = (kQueueLanes + 1) * kQueueStride;

template <int YFMT>
__device__ __forceinline__ float load_sample(const void *y, int64_t idx) {
  if (YFMT == NGDBF_Y_I8) {
    // int8 code y_q; y = y_q / 16 exactly
    return (float)((const int8_t *)y)[idx] * 0.0625f;
  } else {
    return ((const float *)y)[idx];
  }
}

// Saturation at Y_max (Sec. IV-A); ymax <= 0 disables it.  Written as two
// comparisons so that a NaN sample passes through unchanged.
__device__ __forceinline__ float saturate(float v, float ymax) {
  if (ymax > 0.0f) {
    v = (v < -ymax) ? -ymax : v;
    v = (v > ymax) ? ymax : v;
  }
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronisation of the waves that share one frame: the wave itself when a
// single wavefront owns the frame, the workgroup (= the frame) otherwise.
template <int WPF>
__device__ __forceinline__ void frame_sync() {
  if (WPF == 1) {
    wave_sync();
  } else {
    __syncthreads();
  }
}

// The float next above x toward +inf (2^-149 for +-0; +inf and NaN stay).
// With x = fl(r) the exact r is at most next_up(x).
__device__ __forceinline__ float next_up(float x) {
  const uint32_t u = __float_as_uint(x);
  if (!(fabsf(x) < INFINITY)) return x;
  return __uint_as_float(x > 0.0f ? u + 1u : (x < 0.0f ? u - 1u : 1u));
}

// number of set bits of a 64-bit wave mask below this lane
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// g(v) of Sec. IV-E in units of half a quantization step, sign(v) (2L + 1)
// with L = min(floor(|v| c), top); the signum of 0 is 0, NaN stays NaN.
__device__ __forceinline__ float quant_half(float v, float c, float top) {
  if (v == 0.0f) return 0.0f;
  float L = floorf(fabsf(v) * c);
  L = (L > top) ? top : L;
  const float mag = 2.0f * L + 1.0f;
  return v < 0.0f ? -mag : mag;
}

// A sample in the objective's fixed point: rint(2^20 v), clamped to
// +-2^40, NaN counted as 0 (exact in int64).
__device__ __forceinline__ int64_t fixed_sample(float v) {
  float s = v * 0x1p20f;
  s = (s == s) ? s : 0.0f;
  s = (s > 0x1p40f) ? 0x1p40f : s;
  s = (s < -0x1p40f) ? -0x1p40f : s;
  return (int64_t)__builtin_rintf(s);
}

// Key of (E_k, k) for the single-bit argmin: ordered by E, then by k; -0
// counts as +0 (they compare equal).
__device__ __forceinline__ uint64_t argmin_key(float E, int k) {
  uint32_t b = __float_as_uint(E == 0.0f ? 0.0f : E);
  b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)b << 32) | (uint32_t)k;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}

__device__ __forceinline__ float wave_min_f32(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}

// a float as an unsigned key with the same order (-0 just below +0)
__device__ __forceinline__ uint32_t ordered_key(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ordered_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Finish the listed pairs of one wavefront: lanes take entries in turn, draw
// the pair's two Gaussians, and decide E_k < theta_k for both bits, with
// E_k = fmaf(qs, z_k, a_k) (binary32) or a_k + g(qs z_k) (quantized, half
// steps, exact); each owner then reads its two decision bits back.
__device__ __forceinline__ void flush_list(uint32_t *list, int lane, uint32_t total, float qs,
                                           uint32_t pend, uint64_t posb, uint32_t &flip,
                                           bool quant, float qc, float qtop) {
  wave_sync();
  for (uint32_t e = (uint32_t)lane; e < total; e += kWave) {
    uint32_t *ent = list + kEntryWords * e;
    float z0, z1;
    bm_pair(ent[0], ent[1], z0, z1);
    float E0, E1;
    if (quant) {
      E0 = __uint_as_float(ent[2]) + quant_half(qs * z0, qc, qtop);
      E1 = __uint_as_float(ent[3]) + quant_half(qs * z1, qc, qtop);
    } else {
      E0 = __builtin_fmaf(qs, z0, __uint_as_float(ent[2]));
      E1 = __builtin_fmaf(qs, z1, __uint_as_float(ent[3]));
    }
    ent[0] = (E0 < __uint_as_float(ent[4]) ? 1u : 0u) | (E1 < __uint_as_float(ent[5]) ? 2u : 0u);
  }
  wave_sync();
  while (pend) {
    const int q2 = __builtin_ctz(pend);
    pend &= pend - 1;
    const uint32_t ps = (uint32_t)(posb >> (8 * q2)) & 255u;
    const uint32_t bits = list[kEntryWords * ps];
    flip = (flip & ~(3u << (2 * q2))) | (bits << (2 * q2));
  }
  wave_sync();  // the list is refilled next
}

// The same for the base decoder's list: a bit's threshold is theta lambda^u
// with u = t - (its flips so far) (Sec. III-D), looked up here for the listed
// bits only.  Each entry's two decision bits are or-ed into its owner lane's
// decision word at the pair's slot (bits 2q2, 2q2 + 1: the owner's flip bits
// of the pair), which the owner reads once all of the round's entries are
// finished.
__device__ __forceinline__ void flush_list_lazy(uint32_t *list, uint32_t *dec, int lane,
                                                uint32_t first, uint32_t total, float qs,
                                                const float *thtab,
                                                const uint32_t *fcw, int t, float theta, bool adapt,
                                                bool fc_bytes) {
  wave_sync();
  for (uint32_t e = first + (uint32_t)lane; e < total; e += kWave) {
    const uint32_t *ent = list + kEntryWordsLazy * e;
    float z0, z1;
    bm_pair(ent[0], ent[1], z0, z1);
    const float E0 = __builtin_fmaf(qs, z0, __uint_as_float(ent[2]));
    const float E1 = __builtin_fmaf(qs, z1, __uint_as_float(ent[3]));
    const uint32_t tag = ent[4];
    float th0 = theta, th1 = theta;
    if (adapt) {
      // the pair's flip counts (bits k0, k0 + 1; k0 even)
      const uint32_t k0 = tag & 0xFFFFu;
      int f0, f1;
      if (fc_bytes) {
        const uint32_t fc = fcw[k0 >> 2] >> (8 * (k0 & 3u));
        f0 = (int)(fc & 0xFFu);
        f1 = (int)((fc >> 8) & 0xFFu);
      } else {
        const uint32_t fc = fcw[k0 >> 1];
        f0 = (int)(fc & 0xFFFFu);
        f1 = (int)(fc >> 16);
      }
      th0 = thtab[t - f0];
      th1 = thtab[t - f1];
    }
    const uint32_t bits = (E0 < th0 ? 1u : 0u) | (E1 < th1 ? 2u : 0u);
    if (bits) atomicOr(&dec[(tag >> 16) & 63u], bits << (2 * (tag >> 22)));
  }
  wave_sync();  // the decisions have landed; the list is refilled next
}

// Single-bit rule by bounds: the listed pairs are those with a bit whose E_k
// interval reaches the frame's least upper end; each lane transforms its
// entries and keeps the least (E_k, k) key among their valid bits.
__device__ __forceinline__ void flush_single(const uint32_t *list, int lane, uint32_t total,
                                             float qs, bool quant, float qc, float qtop, int n,
                                             uint64_t &best) {
  wave_sync();
  for (uint32_t e = (uint32_t)lane; e < total; e += kWave) {
    const uint32_t *ent = list + kEntryWords * e;
    float z0, z1;
    bm_pair(ent[0], ent[1], z0, z1);
    const float av0 = __uint_as_float(ent[2]), av1 = __uint_as_float(ent[3]);
    const int k0 = (int)ent[4];
    float E0, E1;
    if (quant) {
      E0 = av0 + quant_half(qs * z0, qc, qtop);
      E1 = av1 + quant_half(qs * z1, qc, qtop);
    } else {
      E0 = __builtin_fmaf(qs, z0, av0);
      E1 = __builtin_fmaf(qs, z1, av1);
    }
    if (k0 < n && E0 == E0) {
      const uint64_t key = argmin_key(E0, k0);
      best = key < best ? key : best;
    }
    if (k0 + 1 < n && E1 == E1) {
      const uint64_t key = argmin_key(E1, k0 + 1);
      best = key < best ? key : best;
    }
  }
  wave_sync();  // the list is refilled next
}

// Edges of check i (N(i)) and of bit k (M(k)) in the LDS tables.
struct Tables {
  const uint16_t *col_idx, *row_idx, *row_ptr, *col_ptr;
  int dv, dc;
  // (indices and degrees are below 2^16: 24-bit multiplies are exact)
  __device__ __forceinline__ int row_begin(int i) const { return dc ? (int)__umul24(i, dc) : row_ptr[i]; }
  __device__ __forceinline__ int row_end(int i) const { return dc ? (int)__umul24(i, dc) + dc : row_ptr[i + 1]; }
  __device__ __forceinline__ int col_begin(int k) const { return dv ? (int)__umul24(k, dv) : col_ptr[k]; }
  __device__ __forceinline__ int col_end(int k) const { return dv ? (int)__umul24(k, dv) + dv : col_ptr[k + 1]; }
};

// Decode kernel.  WPF wavefronts cooperate on one frame; each lane owns QPL
// bit quads j = ft + 64*WPF*r (ft = lane index within the frame).  With
// WPF == 1 a workgroup holds several independent frames, one per wave, and
// the round loop has no workgroup barrier.  The grid is persistent; frames
// come from a per-launch queue (an atomic counter).
//
// Per frame in LDS: s (one bit per check, 1 = unsatisfied), u_k (one byte per
// bit: number of unsatisfied checks among M(k)), the count of unsatisfied
// checks, an x / flip bit row, the round's toggle row and event list.  Per
// wave: the Box-Muller list.  At the frame's start s(0) comes from the bits
// with x_k = -1 toggling their checks, u(0) from a gather over each bit's
// checks.
//
// Round t (Sec. III-B/C/D):
//   stop test on the unsatisfied count;
//   for every owned bit S_k = deg_k - 2 u_k and a_k = fmaf(w, S_k, x_k y_k);
//   one Philox call per quad; a pair of bits whose decision the bound on the
//   Box-Muller radius settles (below) needs no transform; the others are
//   compacted into the wave's list, transformed densely, and finished by
//   their owners with E_k = fmaf(qs, z_k, a_k) < theta_k;
//   each flip xors its checks into the toggle row; the owner of each word of
//   s applies its toggles and lists one event per toggled check; every lane
//   then moves u of the listed checks' bits by +-1 (and the owners the
//   unsatisfied count).
//
// Exactness of the bound.  With m = (a >> 8) + 1 = f 2^e, u1 >= 2^(e-24), so
// the radius is at most sqrt(2 (24 - e) ln 2) (the computed radius exceeds it
// by less than 1e-7 relative), and |z| <= radius since |cos|, |sin| <= 1.
// If a_k - theta_k >= |qs| * bound, every draw gives E_k >= theta_k (fma
// rounding is monotone and theta_k is a float): no flip, and the pair needs
// no transform.  The extended kernels test this on squares with a 4e-5
// relative slack that covers all rounding.  The base kernel compares a_k with
// T_c = next_up(fl(theta_max + B_c)) >= theta_max + B_c exactly, where c =
// clz(a | 1), B_c = next_up(fl(|qs| s_c)) >= |qs| s_c, s_c is the bound for c
// leading zeros with 2e-5 slack and theta_max >= theta_k for every bit (see
// the threshold table below), so a_k >= T_c implies a_k - theta_k >= |qs| *
// bound.  Every other pair goes through the transform.
//
// Wave priorities: the phases of a round run at rising priority in round
// order (head, dense draw-and-settle, Box-Muller list, syndrome update), so
// that a SIMD's waves finish the rounds they have started before starting
// new ones; the single-bit kernel's bound phase and candidate list take the
// same levels, and the packed quantized decoder has the same order without
// a list.
//
// EXT kernels add the other decoders of the paper (EXT = kExtMulti: the
// multi-bit rule with quantization or noise reuse; kExtSingle: Step 3a;
// kExtSwitch: mode switching), each with quantization and noise reuse as
// uniform arguments: the single-bit flip of argmin E_k (Step 3a, a frame-wide
// minimum of (E_k, k) keys), mode switching (the objective of Sec. III-B in
// exact fixed point, summed over the frame each round until it first
// decreases), the quantized decoder of Sec. IV-E / V-A (y, w, q_k and
// theta_k through g, all in half-step units, so E_k is an exact small
// integer) and the noise chain of Sec. V-B (the frame's n + T - 1 samples are
// drawn once into LDS; bit k reads element n - 1 + t - k in round t).

// Occupancy target: four waves per SIMD; the base kernel with two or more
// waves per frame (code tables read through the caches) aims higher, and
// more so when each lane holds fewer quads: five waves at four quads per
// lane (a few registers spill, but the extra wave hides more of the table
// reads: C4000 at (4,4) 396 -> 357 ms, C2048 at (2,4) 199 -> 190 ms on a
// mixed-SNR batch), six at two quads, eight at one.
template <int WPF, int QPL, int EXT>
constexpr int waves_per_simd() {
  return (EXT == kExtNone && WPF >= 2) ? (QPL == 1 ? 8 : (QPL == 2 ? 6 : 5)) : 4;
}

template <int WPF, int QPL, int YFMT, bool TRACE, bool REG, int EXT>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(waves_per_simd<WPF, QPL, EXT>())))
decode_kernel(DecodeArgs a) {
  constexpr bool X = EXT != kExtNone;
  extern __shared__ uint32_t lds[];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int fslot = wave / WPF;                // frame slot within the workgroup
  const int ft = tid - fslot * WPF * kWave;    // lane index within the frame
  constexpr int FT = WPF * kWave;              // lanes per frame
  const int n = a.n, m = a.m;
  const int nq = (n + 3) >> 2;
  const int nbytes = (n + 7) >> 3;
  const int T = a.t_max, W = a.smooth_window;

  // stage the code tables once per workgroup; the base kernel with two or
  // more waves per frame reads them from global memory through the caches
  // instead (a frame is a workgroup there, and the LDS goes to more of them)
  constexpr bool TG = EXT == kExtNone && WPF >= 2;
  if (!TG)
    for (int i = tid; i < a.table_words; i += blockDim.x) lds[i] = a.tables[i];
  const uint16_t *t16 = TG ? (const uint16_t *)a.tables : (const uint16_t *)lds;
  Tables tab;
  tab.col_idx = t16;
  tab.row_idx = t16 + a.off_row;
  tab.row_ptr = t16 + a.off_rowptr;
  tab.col_ptr = t16 + a.off_colptr;
  tab.dv = a.dv;
  tab.dc = a.dc;
  uint32_t *slot = lds + a.slots_off + fslot * a.slot_words;
  uint32_t *sw = slot;                     // [sw_words] syndrome bits
  uint32_t *uw = sw + a.sw_words;          // [uw_words] u_k bytes
  uint32_t *xw = uw + a.uw_words;          // [xw_words] x / output bits
  uint32_t *fw = xw + a.xw_words;          // [xw_words] flip bits (trace)
  uint32_t *cnt = fw + (TRACE ? a.xw_words : 0);  // unsatisfied checks
  uint32_t *evn = cnt + 1;                 // [2] events listed (rounds alternate)
  uint32_t *dl = evn + 2;                  // LZ: [2] change of the unsatisfied count (rounds alternate)
  uint32_t *tw = dl + 2;                   // [sw_words] checks toggled this round
  uint32_t *evl = tw + a.sw_words;         // [event_cap] toggle events
  uint32_t *fcw = slot + a.fc_off;         // LZ: flip counts, four or two bits per word
  // EXT: [0] argmin key, [1] objective sum; the noise stream
  uint64_t *red = (uint64_t *)(slot + a.red_off);
  float *stream = (float *)(slot + a.stream_off);
  uint32_t *list = lds + a.slots_off + a.frames_per_block * a.slot_words + wave * a.list_words;
  // LZ: the wave's decision words follow its list entries; zero until a list
  // entry's decision lands, cleared again by the owner that reads it
  uint32_t *dec = list + kEntryWordsLazy * kListCapLazy;
  const uint32_t lane_tag = (uint32_t)lane << 16;
  const bool quant =
      (EXT == kExtMulti || EXT == kExtSingle || EXT == kExtQuantReuse) && a.quant_bits > 0;
  constexpr bool QR = EXT == kExtQuantReuse;
  // The base decoder keeps no per-bit thresholds.  A bit that has flipped F
  // times in rounds 0 .. t-1 has theta_k = theta lambda^(t - F) (Sec. III-D,
  // by repeated binary32 multiplication, 0 < lambda <= 1); every bit that
  // never flipped has theta_t = theta lambda^t.  Rounding is monotone, so the
  // table theta lambda^u is non-decreasing in u for theta <= 0 and
  // non-increasing for theta > 0: every theta_k is at most theta_max(t) =
  // theta_t (theta <= 0) or theta (theta > 0).  The settle test uses
  // theta_max(t) (conservative); a listed bit's own theta_k comes from the
  // table theta lambda^u (u = 0..T, LDS) and the frame's flip counts.
  constexpr bool LZ = EXT == kExtNone;
  const bool adapt = a.lambda != 1.0f;
  float *thtab = (float *)(lds + a.thr_off);
  if (LZ && adapt && tid == 0) {
    float th = a.theta;
    for (int u = 0; u <= a.t_max; ++u) {
      if (u) th = th * a.lambda;
      thtab[u] = th;
    }
  }
  // LZ: lane c's radius bound sqrt(2 min(c + 1, 24) ln 2) with a relative
  // slack of 2e-5, which covers this computation's own rounding (< 3e-7) and
  // the computed radius's excess over the bound (< 1e-7)
  // (also the single-bit kernel's bound on |qs z_k|, BB)
  constexpr bool BB = EXT == kExtSingle;
  const float s_lane =
      (LZ || BB) ? sqrtf((float)(lane < 23 ? lane + 1 : 24) * 1.3862944f) * 1.00002f : 0.0f;
  // kExtQuantReuse: the quantized thresholds theta~(u) = g(theta lambda^u)
  // (Sec. V-A) for every non-flip count u <= T, theta lambda^u by repeated
  // binary32 multiplication, once per workgroup
  int16_t *qtab = (int16_t *)(lds + a.qtab_off);
  if (QR && tid == 0) {
    float th = a.theta;
    for (int u = 0; u <= a.t_max; ++u) {
      if (u) th = th * a.lambda;
      qtab[u] = (int16_t)quant_half(th, a.qc, a.qtop);
    }
  }
  // kExtQuantReuse: the stream reversed, R[i] = g(q) of element L - 1 - i
  // (int16), zero from i = L to the row's end; a lane reads its quad's four
  // samples from two aligned 8-byte words, shifted by the round's phase
  int16_t *qstream = (int16_t *)(slot + a.stream_off);
  if (LZ) dec[lane] = 0u;
  __syncthreads();

  // Frames are handed out from the launch's queue as they are needed, so that
  // the workgroups finish together however the iteration counts fall.  A
  // taker (a wave, or the workgroup when several waves share a frame) takes
  // runs of queue_chunk frames from counter t % kQueueLanes (frame
  // c + kQueueLanes * i is the i-th frame of counter c); once that counter is
  // spent it moves on to the next, until all of them are.
  __shared__ unsigned long long taken;
  // (the wave index is uniform in the wave; readfirstlane lets the compiler
  // keep the counter index, and the frame index with it, in scalar registers)
  const int taker = __builtin_amdgcn_readfirstlane(
      WPF == 1 ? (int)blockIdx.x * (int)(blockDim.x / kWave) + wave : (int)blockIdx.x);
  int qc = taker % kQueueLanes, spent = 0;
  int64_t next = 0, end = 0;  // the taker's current run, in its counter's numbering
  for (;;) {
    int64_t f = -1;  // the taker's next frame; stays -1 once every counter is spent
    while (spent < kQueueLanes) {
      if (next < end) {
        const int64_t c = (int64_t)qc + (int64_t)kQueueLanes * next++;
        if (c < a.n_frames) {
          f = c;
          break;
        }
        // this counter is spent: go on to the next one
        ++spent;
        qc = qc + 1 == kQueueLanes ? 0 : qc + 1;
        next = end = 0;
      } else {
        const unsigned long long chunk = (unsigned long long)a.queue_chunk;
        unsigned long long *qctr = a.queue + qc * kQueueStride;
        unsigned long long g = 0;
        if (WPF == 1) {
          if (lane == 0) g = atomicAdd(qctr, chunk);
        } else {
          if (tid == 0) taken = atomicAdd(qctr, chunk);
          __syncthreads();
          g = taken;
          __syncthreads();
        }
        next = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(g >> 32)) << 32) |
                         (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)g));
        end = next + (int64_t)chunk;
      }
    }
    if (f < 0) break;
    int64_t fs = f;            // data slot of the frame
    uint64_t frame = a.frame_base + (uint64_t)f;
    uint32_t key0 = a.key0, key1 = a.key1;
    if (a.n_segments > 0) {
      int lo = 0, hi = a.n_segments - 1;  // last segment starting at or before f
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.segments[mid].frame_offset <= f) lo = mid; else hi = mid - 1;
      }
      const ngdbf_segment sg = a.segments[lo];
      fs = sg.first_slot + (f - sg.frame_offset);
      if (fs < 0 || fs >= a.pool_frames) continue;  // outside the pools: skipped
      frame = sg.frame_base + (uint64_t)(f - sg.frame_offset);
      // the segment is the same for every lane of the frame: keep the key scalar
      key0 = __builtin_amdgcn_readfirstlane((uint32_t)sg.seed);
      key1 = __builtin_amdgcn_readfirstlane((uint32_t)(sg.seed >> 32));
    }
    const float sigma_f = a.sigma ? a.sigma[fs] : a.sigma_scalar;
    const float qs = a.eta * sigma_f;  // perturbation std (Sec. III-C)
    // qs^2 * 2 ln 2 with a relative slack of 4e-5 (radius bound, squared),
    // floored at 2^-100 so that the settle test below stays strict: a margin
    // whose square underflows is never taken as settled
    const float bound_c = fmaxf((qs * qs) * 0x1.62e8p+0f, 0x1p-100f);
    // LZ: B_c >= |qs| s_c exactly (a negative sigma draws -qs z, whose
    // magnitude has the same bound), and theta_t of round 0
    const float bcl = (LZ || BB) ? next_up(fabsf(qs) * s_lane) : 0.0f;
    float tht = a.theta;
    // LZ: the frame's Philox counter words (wave-uniform) and the per-lane
    // part of every quad's first rounds, computed once per frame
    const uint32_t fr_lo = __builtin_amdgcn_readfirstlane((uint32_t)frame);
    const uint32_t fr_hi = __builtin_amdgcn_readfirstlane((uint32_t)(frame >> 32));
    PhiloxLane pl[QPL];
    if (LZ) {
#pragma unroll
      for (int r = 0; r < QPL; ++r) pl[r] = philox_lane((uint32_t)(ft + FT * r), fr_lo, fr_hi, key0, key1);
    }

    if (X) {
      // the argmin word starts at "no candidate"
      for (int i = ft; i < a.clear_words; i += FT)
        slot[i] = (i == a.red_off || i == a.red_off + 1 || (BB && i == a.red_off + 2)) ? 0xFFFFFFFFu
                                                                                       : 0u;
      if (QR) {
        // sample idx goes to R[L - 1 - idx]; R[L .. stream_lr - 1] = 0
        const int L = a.stream_len;
        const int nsq = (L + 3) >> 2;
        for (int jq = ft; jq < nsq; jq += FT) {
          const Words4 wd = philox4x32_10((uint32_t)jq, 0xFFFFFFFFu, (uint32_t)frame,
                                          (uint32_t)(frame >> 32), key0, key1);
          float z[4];
          bm_pair(wd.w0, wd.w1, z[0], z[1]);
          bm_pair(wd.w2, wd.w3, z[2], z[3]);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int idx = 4 * jq + b;
            if (idx < L) {
              const int i = L - 1 - idx;
              qstream[i] = (int16_t)quant_half(qs * z[b], a.qc, a.qtop);
            }
          }
        }
        for (int i = L + ft; i < a.stream_lr; i += FT) qstream[i] = 0;
      } else if (a.noise_reuse) {
        // the shift-register chain (Sec. V-B): sample j of the frame's stream
        // is draw j & 3 of quad j >> 2 under the iteration word 0xFFFFFFFF
        const int nsq = (a.stream_len + 3) >> 2;
        for (int jq = ft; jq < nsq; jq += FT) {
          const Words4 wd = philox4x32_10((uint32_t)jq, 0xFFFFFFFFu, (uint32_t)frame,
                                          (uint32_t)(frame >> 32), key0, key1);
          float z[4];
          bm_pair(wd.w0, wd.w1, z[0], z[1]);
          bm_pair(wd.w2, wd.w3, z[2], z[3]);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int idx = 4 * jq + b;
            // four interleaved rows: the lanes of a round read consecutive words
            if (idx < a.stream_len)
              stream[b * a.stream_q + jq] = quant ? quant_half(qs * z[b], a.qc, a.qtop) : z[b];
          }
        }
      }
    } else {
      for (int i = ft; i < a.slot_words; i += FT) slot[i] = 0u;
    }
    frame_sync<WPF>();

    // Step 0, x(0) = sign(y) with y saturated (Sec. III-A, IV-A)
    float yv[QPL * 4], thr[QPL * 4];
    uint32_t X2[QPL * 2];  // smoothing sums, two biased 16-bit halves each
    uint32_t deg4[QPL];    // column degrees, one nibble per bit (irregular codes)
    uint32_t xneg = 0;     // bit 4r+b: x_k = -1 for k = 4 j_r + b
    uint32_t vmask = 0;    // bit 4r+b: k = 4 j_r + b is a bit of the code
    // kExtQuantReuse state, one register per pair of bits (4r+2p, 4r+2p+1):
    // x_k g(y_k), the non-flip count u_k and (irregular codes) the degree
    uint32_t xy2[QPL * 2], u2[QPL * 2], dg2[QPL * 2];
#pragma unroll
    for (int r = 0; r < QPL; ++r) {
      const int j = ft + FT * r;
      uint32_t nib = 0, dg = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int k = 4 * j + b;
        float v = 0.0f;
        if (j < nq && k < n) {
          v = saturate(load_sample<YFMT>(a.y, fs * (int64_t)n + k), a.ymax);
          if (!REG) dg |= (uint32_t)(tab.col_ptr[k + 1] - tab.col_ptr[k]) << (4 * b);
        }
        // quantized decoder: y~_k = g(y_k) in half steps (Sec. IV-E)
        // (LZ: a bit past n gets y = +inf: its margin is +inf, it is settled
        // every round and never flips)
        yv[4 * r + b] = quant ? quant_half(v, a.qc, a.qtop)
                              : ((LZ && !(j < nq && k < n)) ? INFINITY : v);
        // a bit past n gets theta = -inf: its margin is +inf, so it is settled
        // every round, never flips and never reaches the output
        thr[4 * r + b] = (j < nq && k < n) ? a.theta : -INFINITY;
        vmask |= (j < nq && k < n ? 1u : 0u) << (4 * r + b);
        nib |= (v < 0.0f ? 1u : 0u) << b;
        if (QR) {
          // x(0) g(y) = |g(y)|; bits past n and NaN samples never flip
          const float gy = yv[4 * r + b];
          const int xyk = (j < nq && k < n && gy == gy) ? (int)fabsf(gy) : kNeverFlip;
          const int dk = REG ? a.dv : (int)((dg >> (4 * b)) & 15u);
          const int sh = 16 * (b & 1);
          if ((b & 1) == 0) {
            xy2[2 * r + (b >> 1)] = 0u;
            u2[2 * r + (b >> 1)] = 0u;
            dg2[2 * r + (b >> 1)] = 0u;
          }
          xy2[2 * r + (b >> 1)] |= ((uint32_t)xyk & 0xFFFFu) << sh;
          dg2[2 * r + (b >> 1)] |= ((uint32_t)dk & 0xFFFFu) << sh;
        }
      }
      X2[2 * r] = X2[2 * r + 1] = (kXBias << 16) | kXBias;
      deg4[r] = dg;
      xneg |= nib << (4 * r);
    }
    frame_sync<WPF>();

    // s(0), u(0) and the unsatisfied count from x(0).  s(0) is the parity of
    // the bits with x_k = -1 (few), each toggling its checks; u(0) is gathered
    // per bit with consecutive lanes on consecutive bits, so that the edge
    // lists are read in near-contiguous runs.
#pragma unroll
    for (int r = 0; r < QPL; ++r) {
      const int j = ft + FT * r;
      uint32_t nib = (xneg >> (4 * r)) & 15u;
      while (nib) {
        const int k = 4 * j + __builtin_ctz(nib);
        nib &= nib - 1;
        for (int e = tab.col_begin(k), e1 = tab.col_end(k); e < e1; ++e) {
          const int i = tab.row_idx[e];
          atomicXor(&sw[i >> 5], 1u << (i & 31));
        }
      }
    }
    frame_sync<WPF>();
    uint32_t nunsat = 0;
    for (int wd = ft; wd < a.sw_words; wd += FT) nunsat += __builtin_popcount(sw[wd]);
    if (nunsat) atomicAdd(cnt, nunsat);
    uint8_t *ub = (uint8_t *)uw;
    if (REG && (a.dv & 1) == 0 && (a.off_row & 1) == 0) {
      // even degree: bit k's edge list is dv / 2 aligned 32-bit words
      const uint32_t *r32 = (const uint32_t *)tab.row_idx;
      const int dh = a.dv >> 1;
      for (int k = ft; k < n; k += FT) {
        uint32_t uk = 0;
        const int w0 = (int)__umul24(k, dh);
        for (int e = 0; e < dh; ++e) {
          const uint32_t pr = r32[w0 + e];
          const int i0 = (int)(pr & 0xFFFFu), i1 = (int)(pr >> 16);
          uk += ((sw[i0 >> 5] >> (i0 & 31)) & 1u) + ((sw[i1 >> 5] >> (i1 & 31)) & 1u);
        }
        ub[k] = (uint8_t)uk;
      }
    } else {
      for (int k = ft; k < n; k += FT) {
        uint32_t uk = 0;
        for (int e = tab.col_begin(k), e1 = tab.col_end(k); e < e1; ++e) {
          const int i = tab.row_idx[e];
          uk += (sw[i >> 5] >> (i & 31)) & 1u;
        }
        ub[k] = (uint8_t)uk;
      }
    }
    frame_sync<WPF>();

    int t = 0;
    int converged = 0;
    // LZ: every wave of the frame keeps the unsatisfied count itself, adding
    // each round's change once the round has ended (so no wave's update can
    // meet another wave's read of the same round, and the round needs no
    // barrier between its dense phase and its toggles)
    uint32_t unsat_reg =
        LZ ? __builtin_amdgcn_readfirstlane(__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
           : 0u;
    bool mu = true;        // mode switching: multi-bit rounds until f drops
    int64_t f_prev = 0;
    const float weff = quant ? a.wq : a.w;
    for (;; ++t) {
      if (LZ || BB) __builtin_amdgcn_s_setprio(kPrioHead);
      if (QR) __builtin_amdgcn_s_setprio(kPrioPackedHead);
      const uint32_t unsat =
          LZ ? unsat_reg
             : __builtin_amdgcn_readfirstlane(__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
      // smoothing window t = T-W .. T (Sec. III-E)
      if (__builtin_expect(W > 0 && t >= T - W, 0)) {
#pragma unroll
        for (int q = 0; q < QPL * 4; ++q)
          X2[q >> 1] += (((xneg >> q) & 1u) ? 0xFFFFFFFFu : 1u) << (16 * (q & 1));
      }
      if (EXT == kExtSwitch && mu) {
        // f(x(t)) = sum_k x_k y_k + sum_i s_i (Sec. III-B) in fixed point;
        // sum_i s_i = m - 2 (unsatisfied checks)
        int64_t part = 0;
#pragma unroll
        for (int q = 0; q < QPL * 4; ++q) {
          const int64_t yf = fixed_sample(yv[q]);  // 0 past the last bit
          part += ((xneg >> q) & 1u) ? -yf : yf;
        }
        part = wave_sum_i64(part);
        if (lane == 0) atomicAdd((unsigned long long *)&red[1], (unsigned long long)part);
        frame_sync<WPF>();
        const int64_t fx = (int64_t)(*(volatile uint64_t *)&red[1]) +
                           ((int64_t)m - 2 * (int64_t)unsat) * ((int64_t)1 << 20);
        frame_sync<WPF>();
        if (ft == 0) red[1] = 0;
        if (t > 0 && fx < f_prev) mu = false;
        f_prev = fx;
      }
      if (__builtin_expect(unsat == 0, 0)) {
        converged = 1;
        break;
      }
      if (t == T) break;

      // ---- decisions for every owned bit (Steps 2, 3)
      uint32_t flip = 0;     // bit 4r+b: flip in this round
      const bool single = EXT == kExtSingle || (EXT == kExtSwitch && !mu);
      if (QR) {
        __builtin_amdgcn_s_setprio(kPrioPackedDense);
        // E~_k = x_k g(y_k) + g(w) S_k + g(q_k) < theta~(u_k), two bits per
        // register in signed 16-bit lanes (exact: every term is a small integer)
        const short2_t w2 = {(short)a.wq, (short)a.wq};
        const int sbase = a.stream_len - n - t;  // R index of bit 4j's sample is sbase + 4j
#pragma unroll
        for (int r = 0; r < QPL; ++r) {
          const int j = ft + FT * r;
          const int jc = j < nq ? j : nq - 1;
          const uint32_t u4 = uw[jc];
          // samples R[sidx .. sidx + 3] from the aligned words at sidx - ph and
          // sidx - ph + 4 (the phase ph = sbase & 3 is the same for every lane)
          const int sidx = sbase + 4 * jc;
          const int ph = sbase & 3;
          const uint2 *wp = (const uint2 *)(qstream + (sidx - ph));
          const uint2 w0 = wp[0];
          uint2 sv = w0;
          if (ph != 0) {
            const uint2 w1 = wp[1];
            if (ph == 1)
              sv = uint2{__builtin_amdgcn_alignbyte(w0.y, w0.x, 2u), __builtin_amdgcn_alignbyte(w1.x, w0.y, 2u)};
            else if (ph == 2)
              sv = uint2{w0.y, w1.x};
            else
              sv = uint2{__builtin_amdgcn_alignbyte(w1.x, w0.y, 2u), __builtin_amdgcn_alignbyte(w1.y, w1.x, 2u)};
          }
          uint32_t fq = 0;
#pragma unroll
          for (int pp = 0; pp < 2; ++pp) {
            const int i2 = 2 * r + pp;
            // unsatisfied-check counts of the pair, one per 16-bit lane
            const uint32_t up = ((u4 >> (16 * pp)) & 0xFFu) | (((u4 >> (16 * pp + 8)) & 0xFFu) << 16);
            const short2_t dgv = REG ? short2_t{(short)a.dv, (short)a.dv} : as_s2(dg2[i2]);
            const short2_t S2 = dgv - (as_s2(up) << (short)1);
            const short2_t E2 = as_s2(xy2[i2]) + w2 * S2 + as_s2(pp ? sv.y : sv.x);
            const uint32_t uu = u2[i2];
            const short2_t th2 = {qtab[uu & 0xFFFFu], qtab[uu >> 16]};
            // sign of E - theta: 1 where the bit flips
            const uint32_t f2 = (as_u32(E2 - th2) >> 15) & 0x00010001u;
            fq |= ((f2 & 1u) | ((f2 >> 15) & 2u)) << (2 * pp);
            // non-flips count up (Sec. V-A); flips negate x_k g(y_k)
            u2[i2] = uu + (f2 ^ 0x00010001u);
            const uint32_t m = f2 * 0xFFFFu;
            xy2[i2] = as_u32(as_s2(xy2[i2] ^ m) - as_s2(m));
          }
          flip |= fq << (4 * r);
        }
      } else if (X && (single || a.noise_reuse)) {
        // every bit's E_k with its draw: from the chain (Sec. V-B) or from
        // its own Philox quad.  The draw source, the arithmetic and the rule
        // are compile-time inside `direct`, so its unrolled loop carries no
        // uniform branches; the selection below happens once per round.
        auto direct = [&](auto reuse_c, auto quant_c, auto single_c) -> uint64_t {
          constexpr bool kReuse = decltype(reuse_c)::value;
          constexpr bool kQuant = decltype(quant_c)::value;
          constexpr bool kSingle = decltype(single_c)::value;
          uint64_t best = ~0ull;
#pragma unroll
          for (int r = 0; r < QPL; ++r) {
            const int j = ft + FT * r;
            const int jc = j < nq ? j : nq - 1;
            float z4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (!kReuse) {
              const Words4 wd = philox4x32_10((uint32_t)j, (uint32_t)t, (uint32_t)frame,
                                              (uint32_t)(frame >> 32), key0, key1);
              bm_pair(wd.w0, wd.w1, z4[0], z4[1]);
              bm_pair(wd.w2, wd.w3, z4[2], z4[3]);
            }
            const uint32_t u4 = uw[jc];
            // bit 4j + b holds element n - 1 + t - 4j - b of the stream in
            // round t; the four rows interleave it (sample i at row i & 3)
            const int c0 = n - 1 + t - 4 * j;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const int q = 4 * r + b;
              const int k = 4 * j + b;
              const bool valid = (vmask >> q) & 1u;
              const float degf = REG ? (float)a.dv : (float)((deg4[r] >> (4 * b)) & 15u);
              const float Sf = __builtin_fmaf(-2.0f, (float)((u4 >> (8 * b)) & 255u), degf);
              const float xy = __uint_as_float(__float_as_uint(yv[q]) ^ (((xneg >> q) & 1u) << 31));
              const float av = __builtin_fmaf(weff, Sf, xy);
              float E;
              if (kReuse) {
                const int idx = c0 - b;
                const float v = valid ? stream[(idx & 3) * a.stream_q + (idx >> 2)] : 0.0f;
                E = kQuant ? av + v : __builtin_fmaf(qs, v, av);
              } else {
                E = kQuant ? av + quant_half(qs * z4[b], a.qc, a.qtop) : __builtin_fmaf(qs, z4[b], av);
              }
              if (kSingle) {
                // Step 3a: the least E_k, ties to the lowest k, NaN never chosen
                const uint64_t key = argmin_key(E, k);
                if (valid && E == E && key < best) best = key;
              } else {
                const float th = (kQuant && thr[q] != -INFINITY) ? quant_half(thr[q], a.qc, a.qtop) : thr[q];
                flip |= (E < th ? 1u : 0u) << q;
              }
            }
          }
          return best;
        };
        // Step 3a by bounds (BB, per-bit draws): with c = clz(a | 1) of the
        // pair's first word, |qs z_k| <= B_c (|g(qs z_k)| <= N_Q - 1 half
        // steps, quantized), so E_k lies in [fl(a_k - B), fl(a_k + B)] (fma
        // and sum round monotonically).  A bit whose lower end exceeds the
        // least upper end U over the frame has E_k > U >= min E: it is neither
        // the argmin nor tied with it.  Only pairs with a bit at or below U go
        // through the transform.
        auto bound_single = [&](auto quant_c) -> uint64_t {
          constexpr bool kQuant = decltype(quant_c)::value;
          __builtin_amdgcn_s_setprio(kPrioDense);
          Words4 wq[QPL];
          float avq[QPL * 4];
          float ub = INFINITY;
#pragma unroll
          for (int r = 0; r < QPL; ++r) {
            const int j = ft + FT * r;
            const int jc = j < nq ? j : nq - 1;
            wq[r] = philox4x32_10((uint32_t)j, (uint32_t)t, (uint32_t)frame, (uint32_t)(frame >> 32),
                                  key0, key1);
            const uint32_t u4 = uw[jc];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              const uint32_t wa = p ? wq[r].w2 : wq[r].w0;
              const float bqp = kQuant ? a.qbound
                                     : __int_as_float(__builtin_amdgcn_ds_bpermute(
                                           __builtin_clz(wa | 1u) << 2, __float_as_int(bcl)));
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int b = 2 * p + h;
                const int q = 4 * r + b;
                const float degf = REG ? (float)a.dv : (float)((deg4[r] >> (4 * b)) & 15u);
                const float Sf = __builtin_fmaf(-2.0f, (float)((u4 >> (8 * b)) & 255u), degf);
                const float xy = __uint_as_float(__float_as_uint(yv[q]) ^ (((xneg >> q) & 1u) << 31));
                const float av = __builtin_fmaf(weff, Sf, xy);
                avq[q] = av;
                if ((vmask >> q) & 1u) ub = fminf(ub, av + bqp);
              }
            }
          }
          ub = wave_min_f32(ub);
          if (WPF > 1) {
            uint32_t *ubw = (uint32_t *)&red[1];
            if (lane == 0) atomicMin(ubw, ordered_key(ub));
            frame_sync<WPF>();
            ub = ordered_value(__hip_atomic_load(ubw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            frame_sync<WPF>();
            if (ft == 0) *ubw = 0xFFFFFFFFu;
          }
          uint64_t bl = ~0ull;
          uint32_t total = 0;
#pragma unroll
          for (int r = 0; r < QPL; ++r) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              // a pair adds at most 64 entries
              if (total > (uint32_t)(kListCap - kWave)) {
                flush_single(list, lane, total, qs, kQuant, a.qc, a.qtop, n, bl);
                total = 0;
              }
              const int q0 = 4 * r + 2 * p;
              const uint32_t wa2 = p ? wq[r].w2 : wq[r].w0;
              const float bqp = kQuant ? a.qbound
                                     : __int_as_float(__builtin_amdgcn_ds_bpermute(
                                           __builtin_clz(wa2 | 1u) << 2, __float_as_int(bcl)));
              const float lo0 = avq[q0] - bqp, lo1 = avq[q0 + 1] - bqp;
              const bool cand = (((vmask >> q0) & 1u) && lo0 <= ub) || (((vmask >> (q0 + 1)) & 1u) && lo1 <= ub);
              const uint64_t bal = __ballot(cand);
              if (cand) {
                uint32_t *ent = list + kEntryWords * (total + mask_rank(bal));
                ent[0] = p ? wq[r].w2 : wq[r].w0;
                ent[1] = p ? wq[r].w3 : wq[r].w1;
                ent[2] = __float_as_uint(avq[q0]);
                ent[3] = __float_as_uint(avq[q0 + 1]);
                ent[4] = (uint32_t)(4 * (ft + FT * r) + 2 * p);
              }
              total += (uint32_t)__popcll(bal);
            }
          }
          __builtin_amdgcn_s_setprio(kPrioList);
          if (total) flush_single(list, lane, total, qs, kQuant, a.qc, a.qtop, n, bl);
          return bl;
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        uint64_t best = ~0ull;
        if (single) {
          if (a.noise_reuse) best = quant ? direct(T_{}, T_{}, T_{}) : direct(T_{}, F_{}, T_{});
          else if (BB) best = quant ? bound_single(T_{}) : bound_single(F_{});
          else best = quant ? direct(F_{}, T_{}, T_{}) : direct(F_{}, F_{}, T_{});
        } else {
          (void)(quant ? direct(T_{}, T_{}, F_{}) : direct(T_{}, F_{}, F_{}));
        }
        if (single) {
          best = wave_min_u64(best);
          if (lane == 0 && best != ~0ull) atomicMin((unsigned long long *)&red[0], (unsigned long long)best);
          frame_sync<WPF>();
          const uint64_t win = *(volatile uint64_t *)&red[0];
          frame_sync<WPF>();
          if (ft == 0) red[0] = ~0ull;
          if (win != ~0ull) {
            const int kb = (int)(uint32_t)win;
            const int jb = kb >> 2;
            if (jb % FT == ft) flip = 1u << (4 * (jb / FT) + (kb & 3));
          }
        }
      } else {
        // LZ: the list holds five words per pair and is finished with the
        // thresholds looked up; otherwise six words with theta_k in them
        constexpr uint32_t kCap = LZ ? (uint32_t)kListCapLazy : (uint32_t)kListCap;
        constexpr int kEW = LZ ? kEntryWordsLazy : kEntryWords;
        // (LZ: entries [first, n_listed) of the list)
        auto drain = [&](uint32_t first, uint32_t n_listed, uint32_t pend_, uint64_t posb_) {
          if (LZ && a.stats && lane == 0)
            atomicAdd((unsigned long long *)&a.stats[1], (unsigned long long)(n_listed - first));
          if (LZ)
            flush_list_lazy(list, dec, lane, first, n_listed, qs, thtab, fcw, t, a.theta, adapt,
                            a.fc_bytes != 0);
          else
            flush_list(list, lane, n_listed, qs, pend_, posb_, flip, quant, a.qc, a.qtop);
        };
        // LZ: lane c holds this round's settle threshold for a pair whose
        // first word has c leading zeros, the float above theta_max + B_c,
        // with theta_max the largest threshold a bit can hold in round t:
        // theta_t for theta <= 0, theta itself for theta > 0
        if (LZ) __builtin_amdgcn_s_setprio(kPrioDense);
        const float tl = LZ ? next_up((a.theta > 0.0f ? a.theta : tht) + bcl) : 0.0f;
        const PhiloxRound pr = philox_round((uint32_t)t, fr_lo, key0, key1);
        uint32_t pend = 0;     // bit 2r+p: pair p of quad r waits in the list
        uint64_t posb = 0;     // list slot of each waiting pair, one byte each
        uint32_t total = 0;    // wave-uniform list length
  #pragma unroll
        for (int r = 0; r < QPL; ++r) {
          // a quad adds at most 2 * 64 entries: drain the list first if needed
          // (LZ: whole passes of 64 from the list's end, keeping the first
          // total mod 64 entries for a later pass, so no pass runs part-empty
          // before the round's last)
          if (r > 0 && __builtin_expect(total > kCap - 2 * kWave, 0)) {
            if (LZ) {
              const uint32_t keep = total & (uint32_t)(kWave - 1);
              drain(keep, total, 0u, 0ull);
              total = keep;
            } else {
              drain(0u, total, pend, posb);
              total = 0;
              pend = 0;
              posb = 0;
            }
          }
          const int j = ft + FT * r;
          // lanes past the last quad run the same code on a clamped index;
          // their margins are +inf (LZ) or their thresholds -inf, so nothing
          // of theirs is ever listed
          const int jc = j < nq ? j : nq - 1;
          const Words4 wd = LZ ? philox_split(pl[r], pr, key0, key1)
                               : philox4x32_10((uint32_t)j, (uint32_t)t, (uint32_t)frame,
                                               (uint32_t)(frame >> 32), key0, key1);
          const uint32_t u4 = uw[jc];
  #pragma unroll
          for (int p = 0; p < 2; ++p) {
            const uint32_t wa = p ? wd.w2 : wd.w0;
            const uint32_t wb = p ? wd.w3 : wd.w1;
            // m = (wa >> 8) + 1 = f 2^e.  clz(wa | 1) + 1 >= 24 - e (equal unless
            // wa >> 8 is 2^i - 1 or wa < 256), so the bound is never smaller
            const int lz = __builtin_clz(wa | 1u);
            float lim = 0.0f, tc = 0.0f;
            if (LZ)
              tc = __int_as_float(__builtin_amdgcn_ds_bpermute(lz << 2, __float_as_int(tl)));
            else
              lim = __builtin_fmaf((float)lz, bound_c, bound_c);
            float avh[2], thh[2];
            bool settled = true;
  #pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int b = 2 * p + h;
              const int q = 4 * r + b;
              // S_k = deg_k - 2 u_k, formed exactly in binary32
              const float degf = REG ? (float)a.dv : (float)((deg4[r] >> (4 * b)) & 15u);
              const float Sf = __builtin_fmaf(-2.0f, (float)((u4 >> (8 * b)) & 255u), degf);
              // x_k y_k: flip the sign bit of y_k when x_k = -1 (exact)
              const float xy = __uint_as_float(__float_as_uint(yv[q]) ^ (((xneg >> q) & 1u) << 31));
              const float av = __builtin_fmaf(weff, Sf, xy);
              avh[h] = av;
              if (!LZ) {
                // quantized: theta~_k = g(theta_k) (Sec. V-A); -inf stays -inf
                const float th = (quant && thr[q] != -INFINITY) ? quant_half(thr[q], a.qc, a.qtop) : thr[q];
                const float mg = av - th;
                thh[h] = th;
                // settled without a draw: a_k - theta_k >= qs * bound (no flip);
                // with lim > 0, mg |mg| >= lim implies mg > 0 (NaN fails the test).
                // Quantized: |g(q_k)| <= N_Q - 1 half steps bounds every draw.
                settled = settled && (quant ? (mg >= a.qbound) : (mg * fabsf(mg) >= lim));
              }
            }
            // LZ: settled without a draw when both a_k >= theta_t + B_c; one
            // comparison of the smaller (a NaN a_k never flips, whichever
            // operand the minimum returns)
            if (LZ) settled = fminf(avh[0], avh[1]) >= tc;
            const uint64_t bal = __ballot(!settled);
            if (!settled) {
              // total <= kCap - 2 * 64 before a quad, so ps < kCap
              const uint32_t ps = total + mask_rank(bal);
              const int q2 = 2 * r + p;
              if (!LZ) {
                pend |= 1u << q2;
                posb |= (uint64_t)(ps & 255u) << (8 * q2);
              }
              uint32_t *ent = list + kEW * ps;
              ent[0] = wa;
              ent[1] = wb;
              ent[2] = __float_as_uint(avh[0]);
              ent[3] = __float_as_uint(avh[1]);
              if (LZ) {
                // the pair's first bit, for its flip counts (a lane past the
                // last quad lists only under a NaN sigma; its bits never
                // flip), the owner lane and the pair's slot
                ent[4] = (uint32_t)(4 * jc + 2 * p) | lane_tag | ((uint32_t)q2 << 22);
              } else {
                ent[4] = __float_as_uint(thh[0]);
                ent[5] = __float_as_uint(thh[1]);
              }
            }
            total += (uint32_t)__popcll(bal);
          }
        }
        if (LZ) __builtin_amdgcn_s_setprio(kPrioList);
        if (total) drain(0u, total, pend, posb);
        if (LZ) {
          // the round's decisions of this lane's listed pairs (0 elsewhere)
          flip = dec[lane];
          dec[lane] = 0u;
        }
      }

      // ---- apply: thresholds (Sec. III-D), decisions, syndrome maintenance
      if (LZ) tht = tht * a.lambda;  // theta_(t+1)
      if (!LZ && !QR && a.lambda != 1.0f && !single) {
#pragma unroll
        for (int q = 0; q < QPL * 4; ++q)
          if (!((flip >> q) & 1u)) thr[q] = thr[q] * a.lambda;
      }
      xneg ^= flip;
      if (LZ || BB) __builtin_amdgcn_s_setprio(kPrioSyndrome);
      if (QR) __builtin_amdgcn_s_setprio(kPrioPackedSyndrome);
      if (TRACE) {
#pragma unroll
        for (int r = 0; r < QPL; ++r) {
          const int j = ft + FT * r;
          const uint32_t nib = (flip >> (4 * r)) & 15u;
          if (j < nq && nib) atomicOr(&fw[j >> 3], nib << (4 * (j & 7)));
        }
      }
      // every wave has read the count before an owner updates it (LZ keeps
      // its count per wave and needs no barrier here)
      if (!LZ) frame_sync<WPF>();
      // 1. each flip toggles s_i of its checks: collect the round's toggles in
      //    a bit row (no atomic result is waited for)
      uint32_t *evc = evn + (t & 1);
      if (ft == 0) evn[(t + 1) & 1] = 0u;  // the next round's event counter
      uint32_t fl = flip;
      while (fl) {
        const int q = __builtin_ctz(fl);
        fl &= fl - 1;
        const int k = 4 * (ft + FT * (q >> 2)) + (q & 3);
        if (LZ && adapt) {
          if (a.fc_bytes)
            atomicAdd(&fcw[k >> 2], 1u << (8 * (k & 3)));
          else
            atomicAdd(&fcw[k >> 1], 1u << (16 * (k & 1)));
        }
        const int c0 = REG ? (int)__umul24(k, a.dv) : tab.col_ptr[k];
        if (REG && a.dv == 3) {
          // the common column weight, unrolled (a wave-uniform branch)
          const int i0 = tab.row_idx[c0], i1 = tab.row_idx[c0 + 1], i2 = tab.row_idx[c0 + 2];
          atomicXor(&tw[i0 >> 5], 1u << (i0 & 31));
          atomicXor(&tw[i1 >> 5], 1u << (i1 & 31));
          atomicXor(&tw[i2 >> 5], 1u << (i2 & 31));
        } else {
          const int c1 = REG ? c0 + a.dv : tab.col_ptr[k + 1];
          for (int e = c0; e < c1; ++e) {
            const int i = tab.row_idx[e];
            atomicXor(&tw[i >> 5], 1u << (i & 31));
          }
        }
      }
      frame_sync<WPF>();
      // LZ: the next round's count-change word (last read at this round's
      // start, before every wave reached the barrier above)
      if (LZ && ft == 0) dl[(t + 1) & 1] = 0u;
      // LZ, one wave per frame: a round without flips has no syndrome update
      // (frames of several waves would need one more exchange to agree on
      // that, which costs more than the update it saves)
      const bool any_flip = !(LZ && WPF == 1) || __builtin_amdgcn_ballot_w64(flip != 0u) != 0ull;
      if (any_flip) {
      // 2. the owner lane of each byte of s (eight checks) applies its
      //    toggles and lists one event (i, +-1) per toggled check, its slots
      //    taken with a single counter update (owner lanes update the counter
      //    at the same time).  A word's four owners are adjacent lanes of one
      //    wave: all four read the word before the first clears it, and each
      //    writes back only its own byte of s.
      //    Rounds that start with many unsatisfied checks (many flips) list
      //    nothing: each owner applies its events' d_c updates of u itself,
      //    which then costs less than listing and spreading them (the
      //    choice is uniform over the frame: every wave holds the same count).
      const uint32_t ecap = (uint32_t)a.event_cap;
      const bool listing = REG && ecap && unsat <= a.list_unsat_max;
      int32_t dcnt = 0;
      for (int bt = ft; bt < 4 * a.sw_words; bt += FT) {
        const int wd = bt >> 2;
        const int sh = 8 * (bt & 3);
        const uint32_t tword = tw[wd];
        if ((bt & 3) == 0 && tword) tw[wd] = 0u;
        const uint32_t tg = (tword >> sh) & 255u;
        if (!tg) continue;
        const uint32_t sn = ((sw[wd] >> sh) & 255u) ^ tg;
        reinterpret_cast<uint8_t *>(sw)[bt] = (uint8_t)sn;
        dcnt += 2 * __builtin_popcount(sn & tg) - __builtin_popcount(tg);
        // event (check i, +-1) applied here: d_c updates of u
        auto apply = [&](int i, bool unsat_now, bool unrolled) {
          const uint32_t d = unsat_now ? 1u : 0xFFFFFFFFu;
          const int r0 = tab.row_begin(i);
          if (unrolled) {
            int k2[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) k2[j] = tab.col_idx[r0 + j];
#pragma unroll
            for (int j = 0; j < 6; ++j) atomicAdd(&uw[k2[j] >> 2], d << (8 * (k2[j] & 3)));
          } else {
            const int r1 = tab.row_end(i);
            for (int e2 = r0; e2 < r1; ++e2) {
              const int k2 = tab.col_idx[e2];
              atomicAdd(&uw[k2 >> 2], d << (8 * (k2 & 3)));
            }
          }
        };
        uint32_t bits = tg;
        if (listing) {
          uint32_t slotn = atomicAdd(evc, (uint32_t)__builtin_popcount(tg));
          while (bits) {
            const int bb = __builtin_ctz(bits);
            bits &= bits - 1;
            const int i = 8 * bt + bb;
            const bool unsat_now = ((sn >> bb) & 1u) != 0u;
            if (__builtin_expect(slotn < ecap, 1))
              evl[slotn] = ((uint32_t)i << 1) | (unsat_now ? 0u : 1u);
            else
              apply(i, unsat_now, false);  // list full: apply the event here
            ++slotn;
          }
        } else if (REG && a.dc == 6) {
          // no list, the common row weight: unrolled (a wave-uniform branch)
          while (bits) {
            const int bb = __builtin_ctz(bits);
            bits &= bits - 1;
            apply(8 * bt + bb, ((sn >> bb) & 1u) != 0u, true);
          }
        } else {
          // no list, or an irregular code
          while (bits) {
            const int bb = __builtin_ctz(bits);
            bits &= bits - 1;
            apply(8 * bt + bb, ((sn >> bb) & 1u) != 0u, false);
          }
        }
      }
      if (dcnt) atomicAdd(LZ ? &dl[t & 1] : cnt, (uint32_t)dcnt);
      if (listing) {
        // 3. every listed event moves u of its check's d_c bits, spread over
        //    all lanes of the frame
        frame_sync<WPF>();
        const uint32_t nev = __hip_atomic_load(evc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint32_t listed = nev < (uint32_t)a.event_cap ? nev : (uint32_t)a.event_cap;
        const uint32_t nup = listed * (uint32_t)a.dc;
        for (uint32_t x = (uint32_t)ft; x < nup; x += FT) {
          // x / d_c, exact here: x < event_cap d_c with event_cap d_c^2 <
          // 2^20 (the reciprocal's error stays below one step) and event_cap
          // < 4096 (x ceil(2^20 / d_c) stays below 2^32); factors below 2^24
          const uint32_t e = __umul24(x, a.dc_recip) >> 20;
          const uint32_t ev = evl[e];
          const int i = (int)(ev >> 1);
          const uint32_t d = (ev & 1u) ? 0xFFFFFFFFu : 1u;
          const int k2 = tab.col_idx[(int)__umul24(i, a.dc) + (int)(x - __umul24(e, a.dc))];
          atomicAdd(&uw[k2 >> 2], d << (8 * (k2 & 3)));
        }
      }
      frame_sync<WPF>();
      // LZ: this round's change of the count (its word was cleared in the
      // previous round, after every wave had read it), then the other word
      // is cleared for the next round
      if (LZ) unsat_reg += __builtin_amdgcn_readfirstlane(__hip_atomic_load(&dl[t & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
      }  // any_flip
      if (TRACE) {
        uint8_t *row = a.trace + ((size_t)f * (size_t)T + (size_t)t) * (size_t)nbytes;
        const uint8_t *fb = (const uint8_t *)fw;
        for (int bb = ft; bb < nbytes; bb += FT) row[bb] = fb[bb];
        frame_sync<WPF>();
        for (int i = ft; i < a.xw_words; i += FT) fw[i] = 0u;
        frame_sync<WPF>();
      }
    }

    // the stats: pairs evaluated (the transformed ones are counted per round)
    if (LZ && a.stats && ft == 0)
      atomicAdd((unsigned long long *)&a.stats[0], (unsigned long long)t * (unsigned long long)((n + 1) / 2));

    // output: x, or sign(X) when T was reached with smoothing on (Sec. III-E)
    for (int i = ft; i < a.xw_words; i += FT) xw[i] = 0u;
    frame_sync<WPF>();
#pragma unroll
    for (int r = 0; r < QPL; ++r) {
      const int j = ft + FT * r;
      uint32_t nib = (xneg >> (4 * r)) & 15u;
      if (!converged && W > 0) {
        nib = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t half = (X2[2 * r + (b >> 1)] >> (16 * (b & 1))) & 0xFFFFu;
          nib |= (half < kXBias ? 1u : 0u) << b;
        }
      }
      if (j < nq && nib) atomicOr(&xw[j >> 3], nib << (4 * (j & 7)));
    }
    frame_sync<WPF>();
    uint8_t *ob = a.out_bits + (size_t)fs * (size_t)nbytes;
    const uint8_t *xb = (const uint8_t *)xw;
    for (int bb = ft; bb < nbytes; bb += FT) ob[bb] = xb[bb];
    if (ft == 0) {
      a.out_iters[fs] = t;
      if (a.out_conv) a.out_conv[fs] = (uint8_t)converged;
    }
    frame_sync<WPF>();  // the slot is cleared for the next frame
  }
  // every taker has taken its last index; the last one to get here empties
  // the queue for the next launch (the others' increments have returned)
  if (WPF == 1 ? lane == 0 : tid == 0) {
    const unsigned long long takers =
        WPF == 1 ? (unsigned long long)gridDim.x * (blockDim.x / kWave) : (unsigned long long)gridDim.x;
    if (atomicAdd(&a.queue[kQueueLanes * kQueueStride], 1ull) == takers - 1) {
      for (int c = 0; c < kQueueLanes; ++c) atomicExch(&a.queue[c * kQueueStride], 0ull);
      atomicExch(&a.queue[kQueueLanes * kQueueStride], 0ull);
    }
  }
}

}  // namespace ngdbf
