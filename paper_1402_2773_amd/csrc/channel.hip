// channel.hip -- the synthetic channel of Sec. III-A and the Monte Carlo
// counters of Sec. IV-A/B on the device (kernels and their C entries).
//
// Channel: y_k = fmaf(sigma_f, z_k, c_hat_k) with c_hat_k = 1 - 2 c_k (BPSK,
// the all-zero codeword unless sent bits are given) and z_k the standard-
// normal draw of bit k from the decoder's own generator (Philox4x32-10 and
// Box-Muller, noise.h) under the iteration word 0xFFFFFFFE, which no decoding
// round (t <= 65535) and not the noise-reuse stream (0xFFFFFFFF) uses, and
// the channel's own key.  int8 storage: y_q = clamp(rint(16 y), -127, 127).
//
// Counters: per frame the bit errors e_f of the decision against the sent
// word, and the frame's iteration count and stop flag, summed over frames:
// bit errors, their squares (for intervals clustered by frame), frame
// errors, undetected errors (stopped on a wrong codeword), iterations,
// unconverged frames and the iteration histogram.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/ngdbf.h"
#include "noise.h"

namespace ngdbf {

constexpr uint32_t kChannelWord = 0xFFFFFFFEu;

// one thread per bit quad of a frame; grid-stride over frames x quads
template <bool I8>
__global__ void __launch_bounds__(256) channel_kernel(int n, int64_t n_frames, const float *sigma,
                                                     float sigma_scalar, uint32_t k0, uint32_t k1,
                                                     uint64_t frame_base, const uint8_t *cw, void *y) {
  const int nq = (n + 3) >> 2;
  const int nb = (n + 7) >> 3;
  const int64_t total = n_frames * (int64_t)nq;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int64_t f = g / nq;
    const int j = (int)(g - f * nq);
    const uint64_t frame = frame_base + (uint64_t)f;
    const float sg = sigma ? sigma[f] : sigma_scalar;
    const Words4 w = philox4x32_10((uint32_t)j, kChannelWord, (uint32_t)frame, (uint32_t)(frame >> 32), k0, k1);
    float z[4];
    bm_pair(w.w0, w.w1, z[0], z[1]);
    bm_pair(w.w2, w.w3, z[2], z[3]);
    const uint32_t cbits = cw ? (uint32_t)(cw[f * nb + (j >> 1)] >> (4 * (j & 1))) : 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int k = 4 * j + b;
      if (k < n) {
        const float v = __builtin_fmaf(sg, z[b], ((cbits >> b) & 1u) ? -1.0f : 1.0f);
        if (I8) {
          float q = __builtin_rintf(16.0f * v);  // 16 v is exact; ties to even
          q = (q >= -127.0f) ? q : -127.0f;      // (a NaN sample saturates low)
          q = (q > 127.0f) ? 127.0f : q;
          ((int8_t *)y)[f * n + k] = (int8_t)q;
        } else {
          ((float *)y)[f * n + k] = v;
        }
      }
    }
  }
}

// one wavefront per frame, grid-stride; counters gathered per workgroup in
// LDS and added to `out` once per workgroup
__global__ void __launch_bounds__(256) frame_stats_kernel(int n, int64_t n_frames, const uint8_t *bits,
                                                          const uint8_t *cw, const int32_t *iters,
                                                          const uint8_t *conv, int t_max, int hist_lds,
                                                          unsigned long long *out) {
  extern __shared__ unsigned long long acc[];  // [6] counters, then [t_max + 1] bins if hist_lds
  unsigned int *hist = (unsigned int *)(acc + 6);
  const int lane = threadIdx.x % 64;
  const int wave = threadIdx.x / 64;
  const int waves = blockDim.x / 64;
  const int bins = t_max + 1;
  for (int i = threadIdx.x; i < 6; i += blockDim.x) acc[i] = 0ull;
  if (hist_lds)
    for (int i = threadIdx.x; i < bins; i += blockDim.x) hist[i] = 0u;
  __syncthreads();
  const int nb = (n + 7) >> 3;
  for (int64_t f = (int64_t)blockIdx.x * waves + wave; f < n_frames; f += (int64_t)gridDim.x * waves) {
    uint32_t e = 0;
    for (int b = lane; b < nb; b += 64) {
      uint32_t d = bits[f * nb + b] ^ (cw ? cw[f * nb + b] : 0u);
      if (b == nb - 1 && (n & 7)) d &= (1u << (n & 7)) - 1u;  // padding bits past n
      e += (uint32_t)__builtin_popcount(d);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
    if (lane == 0) {
      const int it = iters[f];
      const bool stopped = conv ? conv[f] != 0 : true;
      atomicAdd(&acc[0], (unsigned long long)e);
      atomicAdd(&acc[1], (unsigned long long)e * e);
      if (e) atomicAdd(&acc[2], 1ull);
      if (e && conv && stopped) atomicAdd(&acc[3], 1ull);
      atomicAdd(&acc[4], (unsigned long long)(it > 0 ? it : 0));
      if (conv && !stopped) atomicAdd(&acc[5], 1ull);
      const int bin = it < 0 ? 0 : (it > t_max ? t_max : it);
      if (hist_lds)
        atomicAdd(&hist[bin], 1u);
      else
        atomicAdd(&out[6 + bin], 1ull);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 6; i += blockDim.x)
    if (acc[i]) atomicAdd(&out[i], acc[i]);
  if (hist_lds)
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
      if (hist[i]) atomicAdd(&out[6 + i], (unsigned long long)hist[i]);
}

}  // namespace ngdbf

namespace {
int device_cus_now() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}
}  // namespace

namespace ngdbf_host {
int set_error(int code, const char *msg);  // decode.hip: the per-thread message
}

extern "C" {

ngdbf_status ngdbf_channel(int32_t n, int64_t n_frames, const float *sigma, float sigma_scalar,
                           uint64_t seed, uint64_t frame_base, const uint8_t *codewords,
                           int32_t y_format, void *y, void *stream) {
  if (n < 1 || n > 65535) return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "n must be in [1, 65535]");
  if (n_frames < 0) return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "n_frames < 0");
  if (y_format != NGDBF_Y_F32 && y_format != NGDBF_Y_I8)
    return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "unknown y_format");
  if (!sigma && !(sigma_scalar >= 0.0f && sigma_scalar < INFINITY))
    return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "sigma_scalar must be finite and >= 0");
  if (n_frames == 0) return (ngdbf_status)ngdbf_host::set_error(NGDBF_OK, "");
  if (!y) return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "y is required");
  const int64_t quads = n_frames * (int64_t)((n + 3) / 4);
  const int cus = std::max(device_cus_now(), 1);
  const int64_t blocks = std::min<int64_t>((quads + 255) / 256, (int64_t)cus * 16);
  hipStream_t s = (hipStream_t)stream;
  if (y_format == NGDBF_Y_I8)
    hipLaunchKernelGGL(ngdbf::channel_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, n, n_frames,
                       sigma, sigma_scalar, (uint32_t)seed, (uint32_t)(seed >> 32), frame_base, codewords, y);
  else
    hipLaunchKernelGGL(ngdbf::channel_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, n, n_frames,
                       sigma, sigma_scalar, (uint32_t)seed, (uint32_t)(seed >> 32), frame_base, codewords, y);
  if (hipGetLastError() != hipSuccess)
    return (ngdbf_status)ngdbf_host::set_error(NGDBF_EDEVICE, "channel launch failed");
  return (ngdbf_status)ngdbf_host::set_error(NGDBF_OK, "");
}

ngdbf_status ngdbf_frame_stats(int32_t n, int64_t n_frames, const uint8_t *bits,
                               const uint8_t *codewords, const int32_t *iters,
                               const uint8_t *converged, int32_t t_max, int64_t *out,
                               void *stream) {
  if (n < 1 || n > 65535) return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "n must be in [1, 65535]");
  if (n_frames < 0) return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "n_frames < 0");
  if (t_max < 0 || t_max > 65535)
    return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "t_max must be in [0, 65535]");
  if (n_frames == 0) return (ngdbf_status)ngdbf_host::set_error(NGDBF_OK, "");
  if (!bits || !iters || !out)
    return (ngdbf_status)ngdbf_host::set_error(NGDBF_EINVAL, "bits, iters and out are required");
  const int hist_lds = (t_max + 1) <= 8192 ? 1 : 0;
  const size_t lds = 6 * sizeof(unsigned long long) + (hist_lds ? (size_t)(t_max + 1) * 4 : 0);
  const int cus = std::max(device_cus_now(), 1);
  const int64_t blocks = std::min<int64_t>((n_frames + 3) / 4, (int64_t)cus * 8);
  hipLaunchKernelGGL(ngdbf::frame_stats_kernel, dim3((unsigned)blocks), dim3(256), lds, (hipStream_t)stream, n,
                     n_frames, bits, codewords, iters, converged, t_max, hist_lds, (unsigned long long *)out);
  if (hipGetLastError() != hipSuccess)
    return (ngdbf_status)ngdbf_host::set_error(NGDBF_EDEVICE, "statistics launch failed");
  return (ngdbf_status)ngdbf_host::set_error(NGDBF_OK, "");
}

}  // extern "C"
