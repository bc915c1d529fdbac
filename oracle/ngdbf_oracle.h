/*
 * ngdbf_oracle.h -- plain CPU oracle for Noisy Gradient-Descent Bit-Flip
 * (NGDBF) decoding of LDPC codes (Sundararajan, Winstead, Boutillon,
 * IEEE TCOM 2014).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP decoder.
 * Only the test suite, the smoke entry point and the benchmark's CPU
 * baseline leg may load it.  It shares no source with the HIP path: the
 * noise generator below is written here from its published definition
 * (Philox4x32-10, Salmon et al., SC'11) and the Box-Muller transform as
 * this project defines it; the HIP side has its own implementation.
 *
 * All arithmetic of the FP32 decoder is plain IEEE binary32 with an explicit
 * fmaf order; the file is compiled with -ffp-contract=off so that the
 * compiler adds no fusion of its own.
 */
#ifndef NGDBF_ORACLE_H
#define NGDBF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Decoder parameters (paper Sec. III-B..III-E, Sec. IV-A). */
typedef struct {
    float w;             /* syndrome weight w (Sec. III-C, Step 2)              */
    float theta;         /* initial inversion threshold theta (Step 0, 3b; the
                            paper takes theta < 0, any finite value decodes) */
    float lambda;        /* threshold adaptation factor, 0 < lambda <= 1;
                            lambda == 1 is the non-adaptive decoder (III-D)     */
    float eta;           /* perturbation scale: std of q_k is eta*sigma (III-C) */
    float ymax;          /* channel saturation Y_max (IV-A); <= 0: no clamp     */
    int32_t t_max;       /* iteration limit T (Step 4)                          */
    int32_t smooth_window; /* 0: off; W > 0: output sign(X_k) with X summed
                              over t = T-W .. T if T is reached (III-E)        */
    int32_t variant;     /* 0: multi-bit flips E_k < theta_k (Step 3b);
                            1: single-bit flip of argmin E_k (Step 3a);
                            2: mode switching: Step 3b until the objective
                               f(x) first decreases, Step 3a after (III-B)    */
    int32_t quant_bits;  /* 0: binary32 arithmetic; Q in [1, 8]: y, w, q_k and
                            theta_k through the Q-bit quantizer g (IV-E, V-A)  */
    int32_t noise_reuse; /* 0: a fresh q_k per bit and round; 1: one new sample
                            per round passed along a shift-register chain,
                            q_k(t) = q_{k-1}(t-1) (V-B)                        */
} ngdbf_ref_params;

/* Philox4x32-10 block function: out = philox(ctr, key). */
void ngdbf_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                             uint32_t out[4]);

/* Natural log of u1 = m * 2^-24 for an integer m in [1, 2^24], returned as
 * rho = sqrt(-2 ln u1) (the Box-Muller radius). */
float ngdbf_ref_rho(uint32_t m);

/* cos and sin of 2*pi*i*2^-24 for an integer i in [0, 2^24). */
void ngdbf_ref_sincos2pi(uint32_t i, float *c, float *s);

/* Box-Muller pair from two Philox words (a, b): z[0] = rho*cos, z[1] = rho*sin. */
void ngdbf_ref_gauss_pair(uint32_t a, uint32_t b, float z[2]);

/* The four standard-normal draws of bit quad j = k >> 2 of frame `frame`
 * at iteration t, under key `seed`. */
void ngdbf_ref_noise_quad(uint64_t seed, uint64_t frame, uint32_t t,
                          uint32_t quad, float z[4]);

/* z[4j .. 4j+3] = the draws of quads quad0 + j, j < n_quads. */
void ngdbf_ref_noise_block(uint64_t seed, uint64_t frame, uint32_t t,
                           uint32_t quad0, uint32_t n_quads, float *z);

/* Batched helpers for exhaustive tests: rho over m = m0 .. m0+count-1 and
 * sincos over i = i0 .. i0+count-1. */
void ngdbf_ref_rho_range(uint32_t m0, uint32_t count, float *out);
void ngdbf_ref_sincos_range(uint32_t i0, uint32_t count, float *c, float *s);

/* Decode n_frames frames with the FP32 (or quantized) decoder.
 *   H: n columns (bits), m rows (checks), CSR row_ptr[m+1], col_idx[nnz].
 *   y: frames x n, float32 (y_format 0) or int8 codes y_q with y = y_q/16
 *      (y_format 1), row-major.
 *   sigma: per-frame channel std (may be NULL, then sigma_scalar is used).
 *   frame_base: global index of frame 0 (noise key).
 *   out_bits: frames x ceil(n/8), decoded bits c_k = (1-x_k)/2, LSB first.
 *   out_iters: frames, completed flip rounds; out_conv: frames, 1 if the
 *   returned word satisfies every check at the stop (may be NULL).
 *   trace: NULL, or frames x t_max x ceil(n/8) flip masks (bit k of round t
 *   set if x_k flipped in round t); rounds not executed are left zero.
 *   n_threads: worker threads over frames (<= 1: run on the calling thread).
 * Returns 0, or -1 on an invalid argument. */
int ngdbf_ref_decode(int32_t n, int32_t m, const int32_t *row_ptr,
                     const int32_t *col_idx, const void *y, int32_t y_format,
                     int64_t n_frames, const float *sigma, float sigma_scalar,
                     const ngdbf_ref_params *p, uint64_t seed,
                     uint64_t frame_base, uint8_t *out_bits,
                     int32_t *out_iters, uint8_t *out_conv, uint8_t *trace,
                     int32_t n_threads);

/* The quantizer of Sec. IV-E in units of half a quantization step:
 * g(v) * N_Q / Y_max = sign(v) (2L + 1), L = min(floor(|v| c), N_Q/2 - 1),
 * c = fl32(N_Q / (2 Y_max)), N_Q = 2^Q.  sign is the signum: g(0) = 0
 * (a zero perturbation adds nothing); NaN gives NaN. */
float ngdbf_ref_quant_half(float v, int32_t q_bits, float c);

/* Threshold adaptation events of Sec. V-A for the quantized decoder: the
 * thresholds theta_k(u) = g(theta lambda^u), u = 0 .. t_max, with theta
 * lambda^u formed by repeated binary32 multiplication; event i is the first
 * u = tau_i at which the quantized value changes (tau_0 = 0).  Writes at most
 * cap events (value in channel units, tau) and returns their number. */
int32_t ngdbf_ref_threshold_events(float theta, float lambda, float ymax,
                                   int32_t q_bits, int32_t t_max,
                                   double *values, int32_t *taus, int32_t cap);

/* The standard-normal sample that the shift-register chain of Sec. V-B puts
 * at bit k in round t: element n - 1 + t - k of the frame's sample stream,
 * whose element j is draw j & 3 of quad j >> 2 under iteration word
 * 0xFFFFFFFF (a value no round index takes). */
float ngdbf_ref_reuse_sample(uint64_t seed, uint64_t frame, int32_t n,
                             uint32_t t, int32_t k);

/* The synthetic channel of Sec. III-A: y_k = fmaf(sigma_f, z_k, 1 - 2 c_k)
 * for frame f (noise index frame_base + f), with z_k the standard-normal draw
 * of bit k under iteration word 0xFFFFFFFE and key `seed`.
 *   sigma: per-frame std (may be NULL: sigma_scalar for all frames).
 *   codewords: frames x ceil(n/8) sent bits c_k, LSB first (NULL: all zero).
 *   y_format 0: float32 y [F][n]; 1: int8 y_q = clamp(rint(16 y), -127, 127).
 * Returns 0, or -1 on an invalid argument. */
int ngdbf_ref_channel(int32_t n, int64_t n_frames, const float *sigma,
                      float sigma_scalar, uint64_t seed, uint64_t frame_base,
                      const uint8_t *codewords, int32_t y_format, void *y);

/* GDBF objective of Sec. III-B, f(x) = sum_k x_k y_k + sum_i s_i, in fixed
 * point: F = sum_k x_k Y_k + 2^20 sum_i s_i with Y_k = rint(2^20 y_k) (y_k
 * saturated at ymax as in decoding, clamped to +-2^40; NaN counts 0), exact
 * in int64.  x is given as packed decoded bits (frames x ceil(n/8)). */
int ngdbf_ref_objective(int32_t n, int32_t m, const int32_t *row_ptr,
                        const int32_t *col_idx, const void *y, int32_t y_format,
                        int64_t n_frames, float ymax, const uint8_t *bits,
                        int64_t *out);

/* Same algorithm in binary64 arithmetic, with the Gaussian draws formed in
 * double from the same Philox words (statistical comparison only; this is
 * not bit-compatible with the FP32 decoder). y is float32. */
int ngdbf_ref_decode_f64(int32_t n, int32_t m, const int32_t *row_ptr,
                         const int32_t *col_idx, const float *y,
                         int64_t n_frames, const float *sigma,
                         float sigma_scalar, const ngdbf_ref_params *p,
                         uint64_t seed, uint64_t frame_base,
                         uint8_t *out_bits, int32_t *out_iters,
                         uint8_t *out_conv, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
