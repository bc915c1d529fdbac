// probe.hip -- vector-ALU issue-rate probe (device code and its C entry).
//
// The decoder is bound by vector-ALU issue.  A gfx950 SIMD issues wave64
// VALU work in 4-clock slots: one instruction per slot, or two at once when
// both are of the dual-issue kinds (binary32 fma / mul / add and the VOP2
// forms of the simple moves, bitwise ops, add_u32 and lshrrev), while a
// transcendental takes two slots.  This probe runs long unrolled chains of
// one instruction so that the benchmark can measure each opcode's issue time
// on the machine it runs on, and check the hardware issue counters against
// it.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "../../include/ngdbf.h"

namespace ngdbf {

constexpr int kProbeChains = 8;
constexpr int kProbeUnroll = 16;
constexpr int kProbeKinds = 28;

// One chain step of probe kind KIND on chain value x (k: a wave-uniform
// operand, since VOP3 encodings take no literal; q: a 64-bit chain value for
// the 64-bit kinds).  Kinds 5 and up are written out so that the compiler
// neither folds a chain of them nor picks another encoding.
template <int KIND>
__device__ __forceinline__ void probe_step(uint32_t &x, float &f, uint64_t &q, uint32_t y,
                                           uint32_t k, uint64_t k64, uint32_t u) {
  if (KIND == 0) {  // 32-bit integer: (x ^ c) + u, one v_xad_u32
    x = (x ^ 0x9E3779B9u) + u;
  } else if (KIND == 1) {  // 64-bit product (v_mad_u64_u32) and a xor
    const uint64_t p = (uint64_t)0xD2511F53u * x;
    x = (uint32_t)(p >> 32) ^ (uint32_t)p;
  } else if (KIND == 2) {  // binary32 fma
    f = __builtin_fmaf(f, 0.999f, 0.001f);
  } else if (KIND == 3) {  // binary32 multiply
    f = f * 0.999f;
  } else if (KIND == 4) {  // transcendental: hardware square root
    f = __builtin_amdgcn_sqrtf(f);
  } else if (KIND == 5) {
    asm volatile("v_xor_b32 %0, 0x9e3779b9, %0" : "+v"(x));
  } else if (KIND == 6) {
    asm volatile("v_lshlrev_b32 %0, 3, %0" : "+v"(x));
  } else if (KIND == 7) {  // the high word of the product feeds the next one
    uint64_t p;
    asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(p) : "v"(x), "s"(k) : "vcc");
    x = (uint32_t)(p >> 32);
  } else if (KIND == 8) {  // xor3
    asm volatile("v_bitop3_b32 %0, %0, %1, %0 bitop3:0x96" : "+v"(x) : "s"(k));
  } else if (KIND == 9) {
    asm volatile("v_and_b32 %0, 0x7ffffffd, %0" : "+v"(x));
  } else if (KIND == 10) {
    asm volatile("v_or_b32 %0, 0x10000, %0" : "+v"(x));
  } else if (KIND == 11) {
    asm volatile("v_mov_b32 %0, %1" : "=v"(x) : "v"(y));
  } else if (KIND == 12) {
    asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(x) : "v"(y), "s"(k64));
  } else if (KIND == 13) {
    asm volatile("v_add_u32 %0, 0x9e3779b9, %0" : "+v"(x));
  } else if (KIND == 14) {
    asm volatile("v_lshrrev_b32 %0, 3, %0" : "+v"(x));
  } else if (KIND == 15) {
    asm volatile("v_bfe_u32 %0, %0, 3, 17" : "+v"(x));
  } else if (KIND == 16) {  // compare into a lane mask
    uint64_t m;
    asm volatile("v_cmp_eq_u32_e64 %0, %1, %2" : "=s"(m) : "v"(x), "s"(k));
  } else if (KIND == 17) {  // binary32 compare into a lane mask
    uint64_t m;
    asm volatile("v_cmp_lt_f32_e64 %0, %1, %2" : "=s"(m) : "v"(f), "s"(k));
  } else if (KIND == 18) {  // one lane to a scalar register
    uint32_t r;
    asm volatile("v_readlane_b32 %0, %1, 5" : "=s"(r) : "v"(x));
  } else if (KIND == 19) {
    asm volatile("v_writelane_b32 %0, %1, 5" : "+v"(x) : "s"(k));
  } else if (KIND == 20) {
    asm volatile("v_mbcnt_lo_u32_b32 %0, %1, %0" : "+v"(x) : "s"(k));
  } else if (KIND == 21) {
    asm volatile("v_ffbh_u32 %0, %0" : "+v"(x));
  } else if (KIND == 22) {
    asm volatile("v_lshl_add_u64 %0, %0, 2, %1" : "+v"(q) : "s"(k64));
  } else if (KIND == 23) {
    asm volatile("v_add3_u32 %0, %0, %1, %0" : "+v"(x) : "s"(k));
  } else if (KIND == 24) {
    asm volatile("v_mad_u32_u24 %0, %0, %1, %0" : "+v"(x) : "s"(k));
  } else if (KIND == 25) {
    asm volatile("v_lshl_add_u32 %0, %0, 3, %1" : "+v"(x) : "s"(k));
  } else if (KIND == 26) {
    asm volatile("v_or3_b32 %0, %0, %1, %0" : "+v"(x) : "s"(k));
  } else {  // 24-bit product (VOP2)
    asm volatile("v_mul_u32_u24 %0, 0x12345, %0" : "+v"(x));
  }
}

template <int KIND>
__global__ void __launch_bounds__(256) issue_probe_kernel(uint32_t *out, int iters) {
  uint32_t v[kProbeChains];
  float f[kProbeChains];
  uint64_t q[kProbeChains];
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t k = __builtin_amdgcn_readfirstlane(0xD2511F53u ^ (uint32_t)iters);
  const uint64_t k64 = ((uint64_t)k << 32) | (k ^ 0x5555u);
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    v[c] = gid * 2654435761u + 97u * (uint32_t)c;
    f[c] = 1.0f + (float)(v[c] & 1023u) * 0.001f;
    q[c] = v[c];
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c)
        probe_step<KIND>(v[c], f[c], q[c], v[(c + 1) % kProbeChains], k, k64, (uint32_t)u);
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c)
    acc ^= v[c] ^ __float_as_uint(f[c]) ^ (uint32_t)q[c] ^ (uint32_t)(q[c] >> 32);
  out[gid] = acc;
}

template <int... K>
__host__ hipError_t launch_issue_probe(int kind, dim3 g, dim3 b, hipStream_t s, uint32_t *out,
                                       int iters, std::integer_sequence<int, K...>) {
  using Launch = void (*)(uint32_t *, int);
  static const Launch table[] = {issue_probe_kernel<K>...};
  hipLaunchKernelGGL(table[kind], g, b, 0, s, out, iters);
  return hipGetLastError();
}

}  // namespace ngdbf

extern "C" ngdbf_status ngdbf_issue_probe(int32_t kind, int32_t blocks, int32_t iters,
                                          uint32_t *out, void *stream) {
  if (kind < 0 || kind >= ngdbf::kProbeKinds || blocks < 1 || iters < 1 || !out) return NGDBF_EINVAL;
  const hipError_t e = ngdbf::launch_issue_probe(kind, dim3((unsigned)blocks), dim3(256),
                                                 (hipStream_t)stream, out, iters,
                                                 std::make_integer_sequence<int, ngdbf::kProbeKinds>{});
  return e == hipSuccess ? NGDBF_OK : NGDBF_EDEVICE;
}
