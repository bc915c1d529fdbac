// decode.hip -- NGDBF decode kernels for gfx950 and the C ABI of ngdbf.h.
//
// Data layout.
//   HBM: y frame-major [F][n] (float32 or int8), sigma [F], outputs
//        out_bits [F][ceil(n/8)], out_iters [F], out_converged [F].
//   Code tables (library-owned, int32, read through L1/L2): N(i) as CSR
//        row_ptr/col_idx and M(k) as CSC col_ptr/row_idx (Sec. III-A).  After
//        a frame's first syndrome they are only touched for flipped bits.
//   LDS per frame: syndrome bits s, per-bit counts u_k of unsatisfied checks,
//        the unsatisfied-check count and an x/flip bit row; per wavefront a
//        small Box-Muller work list.  A few KB per frame, so occupancy is set
//        by registers.
//   Registers: each lane owns QPL bit quads (bits 4j .. 4j+3) and keeps their
//        saturated y_k, thresholds theta_k, smoothing counters and decisions.
//
// Frames are independent (Sec. IV): one wavefront decodes a frame of up to
// 1024 bits with no workgroup barrier in its round loop; longer codes use
// 2 or 4 wavefronts per frame.  Every round runs on chip; HBM sees y once
// and the decoded bits once per frame.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <cstdarg>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/ngdbf.h"
#include "noise.h"

namespace ngdbf {

constexpr int kWave = 64;
// Box-Muller work-list entries per wavefront (pairs whose flip decision the
// radius bound could not settle); past this a lane transforms its own pairs.
constexpr int kListCap = 256;
// a list entry: the pair's two Philox words, a_k and theta_k of both bits
constexpr int kEntryWords = 6;
// check-toggle events per frame and round held for the parallel u update
constexpr int kEventCap = 256;
// smoothing counters are 16-bit halves biased by this value
constexpr uint32_t kXBias = 32768u;

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
  int32_t slot_words;                     // LDS words per frame slot
};

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

// number of set bits of a 64-bit wave mask below this lane
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Finish the listed pairs of one wavefront: lanes take entries in turn, draw
// the pair's two Gaussians, and decide E_k = fmaf(qs, z_k, a_k) < theta_k for
// both bits; each owner then reads its two decision bits back.
__device__ __forceinline__ void flush_list(uint32_t *list, int lane, uint32_t total, float qs,
                                           uint32_t pend, uint64_t posb, uint32_t &flip) {
  wave_sync();
  for (uint32_t e = (uint32_t)lane; e < total; e += kWave) {
    uint32_t *ent = list + kEntryWords * e;
    float z0, z1;
    bm_pair(ent[0], ent[1], z0, z1);
    const float E0 = __builtin_fmaf(qs, z0, __uint_as_float(ent[2]));
    const float E1 = __builtin_fmaf(qs, z1, __uint_as_float(ent[3]));
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

// Edges of check i (N(i)) and of bit k (M(k)) in the LDS tables.
struct Tables {
  const uint16_t *col_idx, *row_idx, *row_ptr, *col_ptr;
  int dv, dc;
  __device__ __forceinline__ int row_begin(int i) const { return dc ? i * dc : row_ptr[i]; }
  __device__ __forceinline__ int row_end(int i) const { return dc ? i * dc + dc : row_ptr[i + 1]; }
  __device__ __forceinline__ int col_begin(int k) const { return dv ? k * dv : col_ptr[k]; }
  __device__ __forceinline__ int col_end(int k) const { return dv ? k * dv + dv : col_ptr[k + 1]; }
};

// Decode kernel.  WPF wavefronts cooperate on one frame; each lane owns QPL
// bit quads j = ft + 64*WPF*r (ft = lane index within the frame).  With
// WPF == 1 a workgroup holds several independent frames, one per wave, and
// the round loop has no workgroup barrier.
//
// Per frame in LDS: s (one bit per check, 1 = unsatisfied), u_k (one byte per
// bit: number of unsatisfied checks among M(k)), the count of unsatisfied
// checks, and an x / flip bit row.  Per wave: the Box-Muller list.
//
// Round t (Sec. III-B/C/D):
//   stop test on the unsatisfied count;
//   for every owned bit S_k = deg_k - 2 u_k and a_k = fmaf(w, S_k, x_k y_k);
//   one Philox call per quad; a pair of bits whose decision the bound on the
//   Box-Muller radius settles (below) needs no transform; the others are
//   compacted into the wave's list, transformed densely, and finished by
//   their owners with E_k = fmaf(qs, z_k, a_k) < theta_k;
//   each flip toggles s_i of its checks with LDS atomics, and each toggle
//   moves u of the check's bits and the unsatisfied count by +-1.
//
// Exactness of the bound.  With m = (a >> 8) + 1 = f 2^e, u1 >= 2^(e-24), so
// the radius is at most sqrt(2 (24 - e) ln 2) (the computed radius exceeds it
// by less than 1e-7 relative), and |z| <= radius since |cos|, |sin| <= 1.
// If a_k - theta_k >= qs * bound, every draw gives E_k >= theta_k (fma
// rounding is monotone and theta_k is a float): no flip, and the pair needs
// no transform.  The test runs on squares with a 4e-5 relative slack that
// covers all rounding.  Every other pair goes through the transform.
template <int WPF, int QPL, int YFMT, bool TRACE, bool REG>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4)))
decode_kernel(DecodeArgs a) {
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

  // stage the code tables once per workgroup
  for (int i = tid; i < a.table_words; i += blockDim.x) lds[i] = a.tables[i];
  const uint16_t *t16 = (const uint16_t *)lds;
  Tables tab;
  tab.col_idx = t16;
  tab.row_idx = t16 + a.off_row;
  tab.row_ptr = t16 + a.off_rowptr;
  tab.col_ptr = t16 + a.off_colptr;
  tab.dv = a.dv;
  tab.dc = a.dc;
  uint32_t *slot = lds + a.table_words + fslot * a.slot_words;
  uint32_t *sw = slot;                     // [sw_words] syndrome bits
  uint32_t *uw = sw + a.sw_words;          // [uw_words] u_k bytes
  uint32_t *xw = uw + a.uw_words;          // [xw_words] x / output bits
  uint32_t *fw = xw + a.xw_words;          // [xw_words] flip bits (trace)
  uint32_t *cnt = fw + (TRACE ? a.xw_words : 0);  // unsatisfied checks
  uint32_t *evn = cnt + 1;                 // events listed this round
  uint32_t *evl = evn + 1;                 // [kEventCap] toggle events
  uint32_t *list = lds + a.table_words + a.frames_per_block * a.slot_words + wave * (kEntryWords * kListCap);
  __syncthreads();

  const int64_t slots_total = (int64_t)gridDim.x * a.frames_per_block;
  for (int64_t f = (int64_t)blockIdx.x * a.frames_per_block + fslot; f < a.n_frames;
       f += slots_total) {
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

    for (int i = ft; i < a.slot_words; i += FT) slot[i] = 0u;
    frame_sync<WPF>();

    // Step 0, x(0) = sign(y) with y saturated (Sec. III-A, IV-A)
    float yv[QPL * 4], thr[QPL * 4];
    uint32_t X2[QPL * 2];  // smoothing sums, two biased 16-bit halves each
    uint32_t deg4[QPL];    // column degrees, one nibble per bit (irregular codes)
    uint32_t xneg = 0;     // bit 4r+b: x_k = -1 for k = 4 j_r + b
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
        yv[4 * r + b] = v;
        // a bit past n gets theta = -inf: its margin is +inf, so it is settled
        // every round, never flips and never reaches the output
        thr[4 * r + b] = (j < nq && k < n) ? a.theta : -INFINITY;
        nib |= (v < 0.0f ? 1u : 0u) << b;
      }
      X2[2 * r] = X2[2 * r + 1] = (kXBias << 16) | kXBias;
      deg4[r] = dg;
      xneg |= nib << (4 * r);
      if (j < nq && nib) atomicOr(&xw[j >> 3], nib << (4 * (j & 7)));
    }
    frame_sync<WPF>();

    // s(0), u(0) and the unsatisfied count from x(0)
    uint32_t nunsat = 0;
    for (int i = ft; i < m; i += FT) {
      const int e0 = tab.row_begin(i), e1 = tab.row_end(i);
      uint32_t v = 0;
      for (int e = e0; e < e1; ++e) {
        const int k = tab.col_idx[e];
        v ^= (xw[k >> 5] >> (k & 31)) & 1u;
      }
      if (v) {
        atomicOr(&sw[i >> 5], 1u << (i & 31));
        ++nunsat;
        for (int e = e0; e < e1; ++e) {
          const int k = tab.col_idx[e];
          atomicAdd(&uw[k >> 2], 1u << (8 * (k & 3)));
        }
      }
    }
    if (nunsat) atomicAdd(cnt, nunsat);
    frame_sync<WPF>();

    int t = 0;
    int converged = 0;
    for (;; ++t) {
      const uint32_t unsat = *(volatile uint32_t *)cnt;
      // smoothing window t = T-W .. T (Sec. III-E)
      if (W > 0 && t >= T - W) {
#pragma unroll
        for (int q = 0; q < QPL * 4; ++q)
          X2[q >> 1] += (((xneg >> q) & 1u) ? 0xFFFFFFFFu : 1u) << (16 * (q & 1));
      }
      if (unsat == 0) {
        converged = 1;
        break;
      }
      if (t == T) break;

      // ---- decisions for every owned bit (Steps 2, 3b)
      uint32_t flip = 0;     // bit 4r+b: flip in this round
      uint32_t pend = 0;     // bit 2r+p: pair p of quad r waits in the list
      uint64_t posb = 0;     // list slot of each waiting pair, one byte each
      uint32_t total = 0;    // wave-uniform list length
#pragma unroll
      for (int r = 0; r < QPL; ++r) {
        // a quad adds at most 2 * 64 entries: drain the list first if needed
        if (r > 0 && total > (uint32_t)(kListCap - 2 * kWave)) {
          flush_list(list, lane, total, qs, pend, posb, flip);
          total = 0;
          pend = 0;
          posb = 0;
        }
        const int j = ft + FT * r;
        // lanes past the last quad run the same code on a clamped index;
        // their thresholds are -inf, so nothing of theirs is ever listed
        const int jc = j < nq ? j : nq - 1;
        const Words4 wd = philox4x32_10((uint32_t)j, (uint32_t)t, (uint32_t)frame,
                                        (uint32_t)(frame >> 32), key0, key1);
        const uint32_t u4 = uw[jc];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const uint32_t wa = p ? wd.w2 : wd.w0;
          const uint32_t wb = p ? wd.w3 : wd.w1;
          // m = (wa >> 8) + 1 = f 2^e.  clz(wa | 1) + 1 >= 24 - e (equal unless
          // wa >> 8 is 2^i - 1 or wa < 256), so the bound is never smaller
          const float lim = __builtin_fmaf((float)__builtin_clz(wa | 1u), bound_c, bound_c);
          float avh[2];
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
            const float av = __builtin_fmaf(a.w, Sf, xy);
            const float mg = av - thr[q];
            avh[h] = av;
            // settled without a draw: a_k - theta_k >= qs * bound (no flip);
            // with lim > 0, mg |mg| >= lim implies mg > 0 (NaN fails the test)
            settled = settled && (mg * fabsf(mg) >= lim);
          }
          const uint64_t bal = __ballot(!settled);
          if (!settled) {
            const uint32_t ps = total + mask_rank(bal);
            const int q2 = 2 * r + p;
            pend |= 1u << q2;
            posb |= (uint64_t)ps << (8 * q2);
            uint32_t *ent = list + kEntryWords * ps;
            ent[0] = wa;
            ent[1] = wb;
            ent[2] = __float_as_uint(avh[0]);
            ent[3] = __float_as_uint(avh[1]);
            ent[4] = __float_as_uint(thr[4 * r + 2 * p]);
            ent[5] = __float_as_uint(thr[4 * r + 2 * p + 1]);
          }
          total += (uint32_t)__popcll(bal);
        }
      }
      if (total) flush_list(list, lane, total, qs, pend, posb, flip);

      // ---- apply: thresholds (Sec. III-D), decisions, syndrome maintenance
      if (a.lambda != 1.0f) {
#pragma unroll
        for (int q = 0; q < QPL * 4; ++q)
          if (!((flip >> q) & 1u)) thr[q] = thr[q] * a.lambda;
      }
      xneg ^= flip;
      if (TRACE) {
#pragma unroll
        for (int r = 0; r < QPL; ++r) {
          const int j = ft + FT * r;
          const uint32_t nib = (flip >> (4 * r)) & 15u;
          if (j < nq && nib) atomicOr(&fw[j >> 3], nib << (4 * (j & 7)));
        }
      }
      frame_sync<WPF>();  // every wave has read u before any toggle lands
      // each flip toggles s_i of its checks; each toggle is an event (i, +-1)
      // for the u of the check's bits, applied below by all lanes at once
      uint32_t fl = flip;
      int32_t dcnt = 0;
      while (fl) {
        const int q = __builtin_ctz(fl);
        fl &= fl - 1;
        const int k = 4 * (ft + FT * (q >> 2)) + (q & 3);
        const int c0 = REG ? k * a.dv : tab.col_ptr[k];
        const int c1 = REG ? c0 + a.dv : tab.col_ptr[k + 1];
        for (int e = c0; e < c1; ++e) {
          const int i = tab.row_idx[e];
          const uint32_t old = atomicXor(&sw[i >> 5], 1u << (i & 31));
          const bool became_unsat = ((old >> (i & 31)) & 1u) == 0u;
          dcnt += became_unsat ? 1 : -1;
          const uint32_t ev = ((uint32_t)i << 1) | (became_unsat ? 0u : 1u);
          const uint32_t slotn = REG ? atomicAdd(evn, 1u) : (uint32_t)kEventCap;
          if (slotn < (uint32_t)kEventCap) {
            evl[slotn] = ev;
          } else {
            // list full (or an irregular code): apply the event here
            const uint32_t d = became_unsat ? 1u : 0xFFFFFFFFu;
            const int r0 = tab.row_begin(i), r1 = tab.row_end(i);
            for (int e2 = r0; e2 < r1; ++e2) {
              const int k2 = tab.col_idx[e2];
              atomicAdd(&uw[k2 >> 2], d << (8 * (k2 & 3)));
            }
          }
        }
      }
      if (dcnt) atomicAdd(cnt, (uint32_t)dcnt);
      if (REG) {
        frame_sync<WPF>();
        const uint32_t nev = *(volatile uint32_t *)evn;
        const uint32_t listed = nev < (uint32_t)kEventCap ? nev : (uint32_t)kEventCap;
        const uint32_t nup = listed * (uint32_t)a.dc;  // one u update per lane
        for (uint32_t x = (uint32_t)ft; x < nup; x += FT) {
          const uint32_t e = (x * a.dc_recip) >> 20;    // x / d_c, exact here
          const uint32_t ev = evl[e];
          const int i = (int)(ev >> 1);
          const uint32_t d = (ev & 1u) ? 0xFFFFFFFFu : 1u;
          const int k2 = tab.col_idx[i * a.dc + (int)(x - e * a.dc)];
          atomicAdd(&uw[k2 >> 2], d << (8 * (k2 & 3)));
        }
        frame_sync<WPF>();
        if (ft == 0) *evn = 0u;
      }
      frame_sync<WPF>();
      if (TRACE) {
        uint8_t *row = a.trace + ((size_t)f * (size_t)T + (size_t)t) * (size_t)nbytes;
        const uint8_t *fb = (const uint8_t *)fw;
        for (int bb = ft; bb < nbytes; bb += FT) row[bb] = fb[bb];
        frame_sync<WPF>();
        for (int i = ft; i < a.xw_words; i += FT) fw[i] = 0u;
        frame_sync<WPF>();
      }
    }

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
}

// ---------------------------------------------------------------- probes

__global__ void probe_radius_kernel(uint32_t start, uint32_t count, float *out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) out[j] = bm_radius(start + j);
}

__global__ void probe_turn_kernel(uint32_t start, uint32_t count, float *co, float *si) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    float c, s;
    bm_turn(start + j, c, s);
    co[j] = c;
    si[j] = s;
  }
}

__global__ void probe_quad_kernel(uint32_t start, uint32_t count, uint64_t frame, uint32_t iter,
                                  uint32_t k0, uint32_t k1, float *out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    const Draw4 d = draw_quad(start + j, iter, frame, k0, k1);
    for (int b = 0; b < 4; ++b) out[4 * (size_t)j + b] = d.z[b];
  }
}

}  // namespace ngdbf

// ==================================================================== host

struct ngdbf_code {
  int32_t n, m, nnz;
  int device;
  uint32_t *d_tables;  // uint16 col_idx | row_idx [| row_ptr | col_ptr], dword padded
  int32_t table_words;
  int32_t off_row, off_rowptr, off_colptr;
  int32_t dv, dc;      // uniform degrees (0 if irregular)
  int32_t max_col_deg, max_row_deg;
  int32_t shape[3];    // fixed launch shape (waves/frame, quads/lane, frames/block), 0 = default
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = '\0';
  return NGDBF_OK;
}

}  // namespace

namespace ngdbf_host {
// message of a failed call of another translation unit (the server runtime)
int set_error(int code, const char *msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}
}  // namespace ngdbf_host

namespace {

// ---------------------------------------------------------------- devices

struct DeviceState {
  int cus = 0;
  std::mutex mu;                      // guards the fork/join pool below
  std::vector<hipStream_t> streams;   // library streams for batched jobs
  std::vector<hipEvent_t> events;     // one per stream, plus the fork event
  hipEvent_t fork = nullptr;
};

DeviceState &device_state(int dev) {
  static std::mutex mu;
  static std::vector<DeviceState *> all;
  std::lock_guard<std::mutex> g(mu);
  if ((int)all.size() <= dev) all.resize(dev + 1, nullptr);
  if (!all[dev]) {
    all[dev] = new DeviceState();  // lives until the process ends
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) all[dev]->cus = p.multiProcessorCount;
  }
  return *all[dev];
}

// ---------------------------------------------------------------- shapes

struct Shape {
  int wpf, qpl, fpb;
  int block() const { return 64 * wpf * fpb; }
};

// (waves per frame, quads per lane) pairs with built kernels
constexpr int kShapes[][2] = {{1, 1}, {1, 2}, {1, 4}, {2, 2}, {2, 4}, {4, 1},
                              {4, 2}, {4, 4}, {8, 1}, {8, 2}, {16, 1}};

bool shape_built(int wpf, int qpl) {
  for (const auto &sh : kShapes)
    if (sh[0] == wpf && sh[1] == qpl) return true;
  return false;
}

size_t slot_words(const ngdbf_code *c, bool trace) {
  return (size_t)((c->m + 31) / 32) + (size_t)((c->n + 3) / 4) +
         (size_t)((c->n + 31) / 32) * (trace ? 2 : 1) + 2 + ngdbf::kEventCap;
}

size_t lds_bytes(const ngdbf_code *c, const Shape &sh, bool trace) {
  return ((size_t)c->table_words + (size_t)sh.fpb * slot_words(c, trace) +
          (size_t)(sh.block() / 64) * ngdbf::kEntryWords * ngdbf::kListCap) * 4;
}

// NGDBF_OK if the shape can decode the code, else an error with a message
int check_shape(const ngdbf_code *c, const Shape &sh, bool trace) {
  const int nq = (c->n + 3) / 4;
  if (!shape_built(sh.wpf, sh.qpl))
    return fail(NGDBF_EUNSUPPORTED, "no kernel for %d waves x %d quads", sh.wpf, sh.qpl);
  if (nq > 64 * sh.wpf * sh.qpl)
    return fail(NGDBF_EINVAL, "%d waves x %d quads hold %d quads, the code has %d", sh.wpf,
                sh.qpl, 64 * sh.wpf * sh.qpl, nq);
  if (sh.wpf > 1 && sh.fpb != 1)
    return fail(NGDBF_EINVAL, "a frame of several waves is a workgroup of its own");
  if (sh.fpb < 1 || sh.block() > 1024)
    return fail(NGDBF_EINVAL, "workgroup of %d threads", sh.block());
  if (lds_bytes(c, sh, trace) > 160 * 1024)
    return fail(NGDBF_EUNSUPPORTED, "shape needs %zu B of LDS", lds_bytes(c, sh, trace));
  return NGDBF_OK;
}

// The code's fixed shape, or the default: the fewest waves per frame, then
// the fewest quads per lane that hold the code; eight single-wave frames per
// workgroup, which then share one copy of the code tables.
int pick_shape(const ngdbf_code *c, bool trace, Shape *out) {
  if (c->shape[0]) {
    *out = Shape{c->shape[0], c->shape[1], c->shape[2]};
    return check_shape(c, *out, trace);
  }
  const int nq = (c->n + 3) / 4;
  for (const auto &sh : kShapes) {
    if (nq <= 64 * sh[0] * sh[1]) {
      Shape cand{sh[0], sh[1], sh[0] == 1 ? 8 : 1};
      while (check_shape(c, cand, trace) != NGDBF_OK && cand.fpb > 1) cand.fpb /= 2;
      if (check_shape(c, cand, trace) == NGDBF_OK) {
        *out = cand;
        return ok();
      }
    }
  }
  return fail(NGDBF_EUNSUPPORTED, "no launch shape fits n = %d", c->n);
}

// ---------------------------------------------------------------- launch

template <int WPF, int QPL, int YFMT, bool TRACE, bool REG>
int launch(const ngdbf::DecodeArgs &a, const Shape &sh, size_t lds_bytes, int dev, hipStream_t s) {
  auto kern = ngdbf::decode_kernel<WPF, QPL, YFMT, TRACE, REG>;
  if (lds_bytes > 64 * 1024 &&
      hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_bytes) != hipSuccess)
    return fail(NGDBF_EUNSUPPORTED, "cannot raise the LDS limit to %zu bytes", lds_bytes);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, sh.block(), lds_bytes) !=
          hipSuccess ||
      per_cu <= 0)
    return fail(NGDBF_EUNSUPPORTED, "kernel does not fit a compute unit (block %d, LDS %zu B)",
                sh.block(), lds_bytes);
  const int cus = std::max(device_state(dev).cus, 1);
  const int64_t blocks_needed = (a.n_frames + sh.fpb - 1) / sh.fpb;
  // persistent grid: the resident capacity, or fewer blocks for small batches
  const int64_t grid = std::min<int64_t>((int64_t)per_cu * cus, blocks_needed);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(sh.block()), lds_bytes, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

template <int YFMT, bool TRACE>
int dispatch(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev, hipStream_t s) {
#define NGDBF_CASE(W_, Q_)                                                         \
  if (sh.wpf == W_ && sh.qpl == Q_)                                                \
    return a.dv ? launch<W_, Q_, YFMT, TRACE, true>(a, sh, lds, dev, s)            \
                : launch<W_, Q_, YFMT, TRACE, false>(a, sh, lds, dev, s);
  NGDBF_CASE(1, 1)
  NGDBF_CASE(1, 2)
  NGDBF_CASE(1, 4)
  NGDBF_CASE(2, 2)
  NGDBF_CASE(2, 4)
  NGDBF_CASE(4, 1)
  NGDBF_CASE(4, 2)
  NGDBF_CASE(4, 4)
  NGDBF_CASE(8, 1)
  NGDBF_CASE(8, 2)
  NGDBF_CASE(16, 1)
#undef NGDBF_CASE
  return fail(NGDBF_EUNSUPPORTED, "no kernel for %d waves x %d quads", sh.wpf, sh.qpl);
}

int check_params(const ngdbf_params *p) {
  if (!p) return fail(NGDBF_EINVAL, "params is NULL");
  if (!(p->w > 0.0f) || !std::isfinite(p->w)) return fail(NGDBF_EINVAL, "w must be finite and > 0");
  if (!std::isfinite(p->theta)) return fail(NGDBF_EINVAL, "theta must be finite");
  if (!(p->lambda > 0.0f && p->lambda <= 1.0f))
    return fail(NGDBF_EINVAL, "lambda must be in (0, 1]");
  if (!(p->eta >= 0.0f) || !std::isfinite(p->eta)) return fail(NGDBF_EINVAL, "eta must be finite and >= 0");
  if (std::isnan(p->ymax)) return fail(NGDBF_EINVAL, "ymax is NaN");
  if (p->t_max < 0 || p->t_max > 65535) return fail(NGDBF_EINVAL, "t_max must be in [0, 65535]");
  if (p->smooth_window < 0) return fail(NGDBF_EINVAL, "smooth_window must be >= 0");
  if (p->smooth_window > 0 && std::min(p->smooth_window, p->t_max) >= 32767)
    return fail(NGDBF_EUNSUPPORTED, "smoothing over more than 32767 rounds");
  if (p->y_format != NGDBF_Y_F32 && p->y_format != NGDBF_Y_I8)
    return fail(NGDBF_EINVAL, "unknown y_format %d", p->y_format);
  return NGDBF_OK;
}

// Everything a launch needs, validated on the host before any device work.
struct Prepared {
  ngdbf::DecodeArgs a;
  Shape sh;
  size_t lds;
  int dev;
  int y_format;
};

int prepare(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
            float sigma_scalar, const ngdbf_params *p, uint64_t seed, uint64_t frame_base,
            uint8_t *out_bits, int32_t *out_iters, uint8_t *out_conv, uint8_t *trace,
            const Shape *force, Prepared *out, const ngdbf_segment *segments = nullptr,
            int32_t n_segments = 0, int64_t pool_frames = -1) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (n_frames < 0) return fail(NGDBF_EINVAL, "n_frames < 0");
  if (n_frames > 0 && (!y || !out_bits || !out_iters))
    return fail(NGDBF_EINVAL, "y, out_bits and out_iters are required");
  if (!sigma && (!(sigma_scalar >= 0.0f) || !std::isfinite(sigma_scalar)))
    return fail(NGDBF_EINVAL, "sigma_scalar must be finite and >= 0");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NGDBF_EDEVICE, "no HIP device");
  if (dev != code->device)
    return fail(NGDBF_EINVAL, "code lives on device %d, current device is %d", code->device, dev);
  Shape sh;
  if (force) {
    sh = *force;
    rc = check_shape(code, sh, trace != nullptr);
  } else {
    rc = pick_shape(code, trace != nullptr, &sh);
  }
  if (rc) return rc;
  const int n = code->n, m = code->m;
  ngdbf::DecodeArgs &a = out->a;
  a.tables = code->d_tables;
  a.table_words = code->table_words;
  a.off_row = code->off_row;
  a.off_rowptr = code->off_rowptr;
  a.off_colptr = code->off_colptr;
  a.dv = code->dv;
  a.dc = code->dc;
  a.n = n;
  a.m = m;
  a.y = y;
  a.n_frames = n_frames;
  a.sigma = sigma;
  a.sigma_scalar = sigma_scalar;
  a.w = p->w;
  a.theta = p->theta;
  a.lambda = p->lambda;
  a.eta = p->eta;
  a.ymax = p->ymax;
  a.t_max = p->t_max;
  a.smooth_window = p->smooth_window;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.frame_base = frame_base;
  a.out_bits = out_bits;
  a.out_iters = out_iters;
  a.out_conv = out_conv;
  a.trace = trace;
  a.segments = segments;
  a.n_segments = n_segments;
  a.pool_frames = pool_frames >= 0 ? pool_frames : n_frames;
  a.frames_per_block = sh.fpb;
  a.sw_words = (m + 31) / 32;
  a.uw_words = (n + 3) / 4;
  a.xw_words = (n + 31) / 32;
  a.slot_words = (int32_t)slot_words(code, trace != nullptr);
  a.dc_recip = code->dc ? (uint32_t)(((1u << 20) + code->dc - 1) / code->dc) : 0u;
  out->sh = sh;
  out->lds = lds_bytes(code, sh, trace != nullptr);
  out->dev = dev;
  out->y_format = p->y_format;
  return ok();
}

int enqueue(const Prepared &pr, hipStream_t s) {
  if (pr.a.n_frames == 0) return ok();
  const bool trace = pr.a.trace != nullptr;
  if (pr.y_format == NGDBF_Y_I8) {
    return trace ? dispatch<NGDBF_Y_I8, true>(pr.sh, pr.a, pr.lds, pr.dev, s)
                 : dispatch<NGDBF_Y_I8, false>(pr.sh, pr.a, pr.lds, pr.dev, s);
  }
  return trace ? dispatch<NGDBF_Y_F32, true>(pr.sh, pr.a, pr.lds, pr.dev, s)
               : dispatch<NGDBF_Y_F32, false>(pr.sh, pr.a, pr.lds, pr.dev, s);
}

int pending_error() {
  // report an earlier asynchronous fault before queueing more work
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "earlier HIP error: %s", hipGetErrorString(e));
  return NGDBF_OK;
}

int decode_common(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                  float sigma_scalar, const ngdbf_params *p, uint64_t seed, uint64_t frame_base,
                  uint8_t *out_bits, int32_t *out_iters, uint8_t *out_conv, uint8_t *trace,
                  void *stream) {
  Prepared pr;
  int rc = prepare(code, y, n_frames, sigma, sigma_scalar, p, seed, frame_base, out_bits,
                   out_iters, out_conv, trace, nullptr, &pr);
  if (rc) return rc;
  rc = pending_error();
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (trace && n_frames > 0 && p->t_max > 0) {
    const size_t tb = (size_t)n_frames * (size_t)p->t_max * (size_t)((code->n + 7) / 8);
    if (hipMemsetAsync(trace, 0, tb, s) != hipSuccess)
      return fail(NGDBF_EDEVICE, "trace clear failed");
  }
  return enqueue(pr, s);
}

}  // namespace

extern "C" {

const char *ngdbf_last_error(void) { return g_err; }

int ngdbf_create_code(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col_idx,
                      ngdbf_code **out) {
  if (!out) return fail(NGDBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!row_ptr || !col_idx) return fail(NGDBF_EINVAL, "row_ptr and col_idx are required");
  if (m < 1 || n <= m || n > 65535) return fail(NGDBF_EINVAL, "need 1 <= m < n <= 65535");
  if (row_ptr[0] != 0) return fail(NGDBF_EINVAL, "row_ptr[0] must be 0");
  for (int i = 0; i < m; ++i) {
    if (row_ptr[i + 1] <= row_ptr[i]) return fail(NGDBF_EINVAL, "row %d is empty or row_ptr decreases", i);
  }
  const int64_t nnz = row_ptr[m];
  if (nnz > (1 << 24)) return fail(NGDBF_EUNSUPPORTED, "nnz %lld exceeds 2^24", (long long)nnz);
  std::vector<int32_t> colcnt(n + 1, 0);
  for (int i = 0; i < m; ++i) {
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int c = col_idx[e];
      if (c < 0 || c >= n) return fail(NGDBF_EINVAL, "col_idx[%d] = %d out of range", e, c);
      for (int e2 = row_ptr[i]; e2 < e; ++e2)
        if (col_idx[e2] == c) return fail(NGDBF_EINVAL, "row %d repeats column %d", i, c);
      colcnt[c + 1]++;
    }
  }
  for (int k = 0; k < n; ++k)
    if (colcnt[k + 1] == 0) return fail(NGDBF_EINVAL, "column %d is empty", k);
  std::vector<int32_t> colptr(n + 1, 0);
  for (int k = 0; k < n; ++k) colptr[k + 1] = colptr[k] + colcnt[k + 1];
  std::vector<int32_t> rowidx(nnz), fill(colptr.begin(), colptr.end() - 1);
  for (int i = 0; i < m; ++i)
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) rowidx[fill[col_idx[e]]++] = i;

  int maxr = 0, maxc = 0, minr = 1 << 30, minc = 1 << 30;
  for (int i = 0; i < m; ++i) {
    maxr = std::max(maxr, row_ptr[i + 1] - row_ptr[i]);
    minr = std::min(minr, row_ptr[i + 1] - row_ptr[i]);
  }
  for (int k = 0; k < n; ++k) {
    maxc = std::max(maxc, colptr[k + 1] - colptr[k]);
    minc = std::min(minc, colptr[k + 1] - colptr[k]);
  }
  if (maxc > 15) return fail(NGDBF_EUNSUPPORTED, "column degree %d exceeds 15", maxc);
  const bool regular = (maxr == minr) && (maxc == minc);
  if (nnz > 65535 && !regular)
    return fail(NGDBF_EUNSUPPORTED, "an irregular code needs nnz <= 65535 (16-bit pointers)");
  // uint16 tables: col_idx | row_idx [| row_ptr | col_ptr]
  std::vector<uint16_t> t16;
  t16.reserve((size_t)(2 * nnz + m + n + 4));
  for (int64_t e = 0; e < nnz; ++e) t16.push_back((uint16_t)col_idx[e]);
  const int off_row = (int)t16.size();
  for (int64_t e = 0; e < nnz; ++e) t16.push_back((uint16_t)rowidx[e]);
  int off_rowptr = 0, off_colptr = 0;
  if (!regular) {
    off_rowptr = (int)t16.size();
    for (int i = 0; i <= m; ++i) t16.push_back((uint16_t)row_ptr[i]);
    off_colptr = (int)t16.size();
    for (int k = 0; k <= n; ++k) t16.push_back((uint16_t)colptr[k]);
  }
  if (t16.size() & 1) t16.push_back(0);
  const int words = (int)(t16.size() / 2);

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NGDBF_EDEVICE, "no HIP device");
  ngdbf_code *c = (ngdbf_code *)calloc(1, sizeof(ngdbf_code));
  if (!c) return fail(NGDBF_ENOMEM, "host allocation failed");
  c->n = n;
  c->m = m;
  c->nnz = (int32_t)nnz;
  c->device = dev;
  c->table_words = words;
  c->off_row = off_row;
  c->off_rowptr = off_rowptr;
  c->off_colptr = off_colptr;
  c->dv = regular ? maxc : 0;
  c->dc = regular ? maxr : 0;
  c->max_row_deg = maxr;
  c->max_col_deg = maxc;
  c->shape[0] = c->shape[1] = c->shape[2] = 0;
  const size_t bytes = (size_t)words * 4;
  if (hipMalloc((void **)&c->d_tables, bytes) != hipSuccess) {
    free(c);
    return fail(NGDBF_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  if (hipMemcpy(c->d_tables, t16.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->d_tables);
    free(c);
    return fail(NGDBF_EDEVICE, "upload of the code tables failed");
  }
  *out = c;
  return ok();
}

int ngdbf_destroy_code(ngdbf_code *code) {
  if (!code) return ok();
  const hipError_t e = hipFree(code->d_tables);
  free(code);
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "hipFree failed: %s", hipGetErrorString(e));
  return ok();
}

int ngdbf_code_info(const ngdbf_code *code, int32_t *n, int32_t *m, int32_t *nnz) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (n) *n = code->n;
  if (m) *m = code->m;
  if (nnz) *nnz = code->nnz;
  return ok();
}

int ngdbf_decode(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                 float sigma_scalar, const ngdbf_params *params, uint64_t seed,
                 uint64_t frame_base, uint8_t *out_bits, int32_t *out_iters,
                 uint8_t *out_converged, void *stream) {
  return decode_common(code, y, n_frames, sigma, sigma_scalar, params, seed, frame_base, out_bits,
                       out_iters, out_converged, nullptr, stream);
}

int ngdbf_decode_trace(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                       float sigma_scalar, const ngdbf_params *params, uint64_t seed,
                       uint64_t frame_base, uint8_t *out_bits, int32_t *out_iters,
                       uint8_t *out_converged, uint8_t *flip_masks, void *stream) {
  if (n_frames > 0 && params && params->t_max > 0 && !flip_masks)
    return fail(NGDBF_EINVAL, "flip_masks is required");
  return decode_common(code, y, n_frames, sigma, sigma_scalar, params, seed, frame_base, out_bits,
                       out_iters, out_converged, flip_masks ? flip_masks : nullptr, stream);
}

int ngdbf_noise_probe(int32_t kind, uint32_t start, uint32_t count, uint64_t seed, uint64_t frame,
                      uint32_t iter, float *out0, float *out1, void *stream) {
  if (count == 0) return ok();
  if (!out0) return fail(NGDBF_EINVAL, "out0 is NULL");
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = (count + 255) / 256;
  if (kind == 0) {
    if (start < 1 || (uint64_t)start + count - 1 > (1ull << 24))
      return fail(NGDBF_EINVAL, "radius probe range must lie in [1, 2^24]");
    hipLaunchKernelGGL(ngdbf::probe_radius_kernel, dim3(blocks), dim3(256), 0, s, start, count, out0);
  } else if (kind == 1) {
    if (!out1) return fail(NGDBF_EINVAL, "out1 is NULL");
    if ((uint64_t)start + count > (1ull << 24))
      return fail(NGDBF_EINVAL, "angle probe range must lie in [0, 2^24)");
    hipLaunchKernelGGL(ngdbf::probe_turn_kernel, dim3(blocks), dim3(256), 0, s, start, count, out0,
                       out1);
  } else if (kind == 2) {
    hipLaunchKernelGGL(ngdbf::probe_quad_kernel, dim3(blocks), dim3(256), 0, s, start, count, frame,
                       iter, (uint32_t)seed, (uint32_t)(seed >> 32), out0);
  } else {
    return fail(NGDBF_EINVAL, "unknown probe kind %d", kind);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "probe launch failed: %s", hipGetErrorString(e));
  return ok();
}

int ngdbf_decode_segments(const ngdbf_code *code, const void *y_pool, const float *sigma_pool,
                          float sigma_scalar, int64_t pool_frames, const ngdbf_params *params,
                          const ngdbf_segment *segments, int32_t n_segments, int64_t n_frames,
                          uint8_t *bits_pool, int32_t *iters_pool, uint8_t *conv_pool,
                          void *stream) {
  if (n_frames > 0 && (n_segments < 1 || !segments))
    return fail(NGDBF_EINVAL, "segments are required");
  if (pool_frames < 0) return fail(NGDBF_EINVAL, "pool_frames < 0");
  Prepared pr;
  int rc = prepare(code, y_pool, n_frames, sigma_pool, sigma_scalar, params, 0, 0, bits_pool,
                   iters_pool, conv_pool, nullptr, nullptr, &pr, segments, n_segments, pool_frames);
  if (rc) return rc;
  rc = pending_error();
  if (rc) return rc;
  return enqueue(pr, (hipStream_t)stream);
}

int ngdbf_code_set_shape(ngdbf_code *code, int32_t waves_per_frame, int32_t quads_per_lane,
                         int32_t frames_per_block) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (!waves_per_frame && !quads_per_lane && !frames_per_block) {
    code->shape[0] = code->shape[1] = code->shape[2] = 0;
    return ok();
  }
  const Shape sh{waves_per_frame, quads_per_lane, frames_per_block};
  int rc = check_shape(code, sh, false);
  if (rc) return rc;
  code->shape[0] = sh.wpf;
  code->shape[1] = sh.qpl;
  code->shape[2] = sh.fpb;
  return ok();
}

int ngdbf_code_get_shape(const ngdbf_code *code, int32_t shape[3]) {
  if (!code || !shape) return fail(NGDBF_EINVAL, "code and shape are required");
  Shape sh;
  int rc = pick_shape(code, false, &sh);
  if (rc) return rc;
  shape[0] = sh.wpf;
  shape[1] = sh.qpl;
  shape[2] = sh.fpb;
  return ok();
}

int ngdbf_autotune(ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                   float sigma_scalar, const ngdbf_params *params, uint64_t seed, int32_t best[3],
                   float *elapsed_ms, void *stream) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (n_frames <= 0) return fail(NGDBF_EINVAL, "autotuning needs a sample of frames");
  int rc = pending_error();
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t nb = (size_t)(code->n + 7) / 8;
  uint8_t *bits = nullptr;
  int32_t *iters = nullptr;
  if (hipMalloc((void **)&bits, (size_t)n_frames * nb) != hipSuccess ||
      hipMalloc((void **)&iters, (size_t)n_frames * 4) != hipSuccess) {
    (void)hipFree(bits);
    return fail(NGDBF_ENOMEM, "autotune scratch of %lld frames", (long long)n_frames);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  Shape best_sh{0, 0, 0};
  float best_ms = 0.0f;
  const int nq = (code->n + 3) / 4;
  for (const auto &ks : kShapes) {
    if (nq > 64 * ks[0] * ks[1]) continue;
    // more quads per lane or waves per frame than the code needs only idle lanes
    if (ks[1] > 1 && nq <= 64 * ks[0] * (ks[1] / 2)) continue;
    if (ks[0] > 1 && nq <= 64 * (ks[0] / 2) * ks[1]) continue;
    for (int fpb : {1, 2, 4, 8, 16}) {
      const Shape cand{ks[0], ks[1], fpb};
      if (check_shape(code, cand, false) != NGDBF_OK) continue;
      Prepared pr;
      rc = prepare(code, y, n_frames, sigma, sigma_scalar, params, seed, 0, bits, iters, nullptr,
                   nullptr, &cand, &pr);
      if (rc) break;
      rc = enqueue(pr, s);  // warm-up
      if (rc == NGDBF_EUNSUPPORTED) {  // rejected before launch (occupancy, LDS)
        rc = NGDBF_OK;
        continue;
      }
      if (rc) break;
      (void)hipEventRecord(e0, s);
      for (int rep = 0; rep < 2 && !rc; ++rep) rc = enqueue(pr, s);
      (void)hipEventRecord(e1, s);
      if (rc) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(NGDBF_EDEVICE, "autotune run failed");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms *= 0.5f;
      if (!best_sh.wpf || ms < best_ms) {
        best_sh = cand;
        best_ms = ms;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(bits);
  (void)hipFree(iters);
  if (rc) return rc;
  if (!best_sh.wpf) return fail(NGDBF_EUNSUPPORTED, "no launch shape fits this code");
  code->shape[0] = best_sh.wpf;
  code->shape[1] = best_sh.qpl;
  code->shape[2] = best_sh.fpb;
  if (best) {
    best[0] = best_sh.wpf;
    best[1] = best_sh.qpl;
    best[2] = best_sh.fpb;
  }
  if (elapsed_ms) *elapsed_ms = best_ms;
  return ok();
}

int ngdbf_decode_batch(const ngdbf_job *jobs, int32_t n_jobs, void *stream) {
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(NGDBF_EINVAL, "bad job array");
  std::vector<Prepared> prs((size_t)n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    const ngdbf_job &j = jobs[i];
    const int rc = prepare(j.code, j.y, j.n_frames, j.sigma, j.sigma_scalar, &j.params, j.seed,
                           j.frame_base, j.out_bits, j.out_iters, j.out_converged, nullptr,
                           nullptr, &prs[i]);
    if (rc) {
      char msg[512];
      snprintf(msg, sizeof msg, "%s", g_err);
      return fail(rc, "job %d: %s", i, msg);
    }
    if (i && prs[i].dev != prs[0].dev) return fail(NGDBF_EINVAL, "jobs span several devices");
  }
  int rc = pending_error();
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n_jobs == 0) return ok();
  if (n_jobs == 1) return enqueue(prs[0], s);
  DeviceState &ds = device_state(prs[0].dev);
  std::lock_guard<std::mutex> g(ds.mu);
  const size_t lanes = (size_t)std::min(n_jobs, 8);
  while (ds.streams.size() < lanes) {
    hipStream_t ns = nullptr;
    hipEvent_t ne = nullptr;
    // default priority: library streams never outrank the caller's work
    if (hipStreamCreateWithFlags(&ns, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ne, hipEventDisableTiming) != hipSuccess)
      return fail(NGDBF_EDEVICE, "cannot create the batch streams");
    ds.streams.push_back(ns);
    ds.events.push_back(ne);
  }
  if (!ds.fork && hipEventCreateWithFlags(&ds.fork, hipEventDisableTiming) != hipSuccess)
    return fail(NGDBF_EDEVICE, "cannot create the fork event");
  // fork: every library stream waits for the work already queued on `stream`
  if (hipEventRecord(ds.fork, s) != hipSuccess) return fail(NGDBF_EDEVICE, "fork record failed");
  for (size_t l = 0; l < lanes; ++l)
    if (hipStreamWaitEvent(ds.streams[l], ds.fork, 0) != hipSuccess)
      return fail(NGDBF_EDEVICE, "fork wait failed");
  for (int i = 0; i < n_jobs; ++i) {
    rc = enqueue(prs[i], ds.streams[(size_t)i % lanes]);
    if (rc) break;
  }
  // join: `stream` waits for every library stream (also after a failure, so
  // that the fork/join structure stays balanced under graph capture)
  for (size_t l = 0; l < lanes; ++l) {
    if (hipEventRecord(ds.events[l], ds.streams[l]) != hipSuccess ||
        hipStreamWaitEvent(s, ds.events[l], 0) != hipSuccess)
      return fail(NGDBF_EDEVICE, "join failed");
  }
  return rc;
}

}  // extern "C"
