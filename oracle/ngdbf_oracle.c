/*
 * ngdbf_oracle.c -- plain CPU oracle for NGDBF decoding.
 *
 * TEST INFRASTRUCTURE ONLY (see ngdbf_oracle.h).  Written for readability:
 * every step follows the paper's order and notation, one frame at a time,
 * with no blocking, fusion or reordering.
 *
 * Paper sections followed:
 *   Sec. III-A  notation: H, N(i), M(k), bipolar x, syndrome s_i, x(0)=sign(y)
 *   Sec. III-B  GDBF Steps 1-4, multi-bit threshold flip (Step 3b)
 *   Sec. III-C  noisy inversion function E_k = x_k y_k + w sum s_i + q_k,
 *               q_k ~ N(0, eta^2 N0/2)
 *   Sec. III-D  adaptive thresholds: theta_k <- theta_k * lambda when x_k is
 *               not flipped
 *   Sec. III-E  output smoothing: X_k += x_k over the last W rounds; output
 *               sign(X_k) when T is reached without convergence
 *   Sec. IV-A   channel saturation at Y_max
 *
 * The paper does not specify its random number generator.  This project's
 * reading: q_k = fl(eta*sigma) * z_k with z_k drawn from Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11) followed by a Box-Muller transform whose log, square root and
 * sine/cosine are fixed sequences of IEEE binary32 operations given below.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 */
#include "ngdbf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 4 "Philox").             */
/* ------------------------------------------------------------------ */

/* Multipliers and Weyl key increments of Philox-4x32 as published. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u /* golden ratio */
#define PHILOX_W1 0xBB67AE85u /* sqrt(3) - 1  */

void ngdbf_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                             uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        /* One Philox S-box: two 32x32->64 products, the high halves mixed
         * with the other two words and the round key, then a word swap. */
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        /* key schedule: add the Weyl constants after each round */
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------ */
/* Box-Muller in binary32.                                            */
/*                                                                    */
/* u1 = m * 2^-24 with m = (a >> 8) + 1 in [1, 2^24]: never 0.        */
/* phi = 2*pi * i * 2^-24 with i = b >> 8 in [0, 2^24).               */
/* z0 = sqrt(-2 ln u1) cos(phi), z1 = sqrt(-2 ln u1) sin(phi).        */
/* ------------------------------------------------------------------ */

/* binary32 constants (each literal is exactly the float it names) */
#define F_SQRT2     0x1.6a09e6p+0f   /* fl(sqrt 2)                        */
#define F_TWO_LN2   0x1.62e430p+0f   /* fl(2 ln 2)                        */
#define F_TWOPI_M24 0x1.921fb6p-22f  /* fl(2 pi) * 2^-24, exact scaling   */

/* Series coefficients, each the binary32 value nearest the rational. */
#define C_1_3       0x1.555556p-2f   /* 1/3        */
#define C_1_5       0x1.99999ap-3f   /* 1/5        */
#define C_1_7       0x1.24924ap-3f   /* 1/7        */
#define C_1_9       0x1.c71c72p-4f   /* 1/9        */
#define C_1_11      0x1.745d18p-4f   /* 1/11       */
#define S_3         -0x1.555556p-3f  /* -1/3!      */
#define S_5         0x1.111112p-7f   /* 1/5!       */
#define S_7         -0x1.a01a02p-13f /* -1/7!      */
#define S_9         0x1.71de3ap-19f  /* 1/9!       */
#define K_2         -0.5f            /* -1/2!      */
#define K_4         0x1.555556p-5f   /* 1/4!       */
#define K_6         -0x1.6c16c2p-10f /* -1/6!      */
#define K_8         0x1.a01a02p-16f  /* 1/8!       */
#define K_10        -0x1.27e4fcp-22f /* -1/10!     */

float ngdbf_ref_rho(uint32_t m) {
    /* ln u1 = (e - 24) ln 2 + ln f with m = f * 2^e, f in [1/sqrt2, sqrt2).
     * ln f = 2 atanh(s), s = (f - 1)/(f + 1), |s| <= 0.1716, by its odd
     * power series truncated after s^11 (remainder < 2e-11).
     * rho^2 = -2 ln u1 = (24 - e) * 2 ln 2 - 4 s P(s^2). */
    int e = 31 - __builtin_clz(m);           /* floor(log2 m), 0..24      */
    float f = ldexpf((float)m, -e);          /* exact, in [1, 2)          */
    if (f > F_SQRT2) {
        f = f * 0.5f;                        /* exact                     */
        e = e + 1;
    }
    float num = f - 1.0f;                    /* exact (Sterbenz)          */
    float den = f + 1.0f;
    float s = num / den;
    float s2 = s * s;
    float p = fmaf(s2, C_1_11, C_1_9);
    p = fmaf(s2, p, C_1_7);
    p = fmaf(s2, p, C_1_5);
    p = fmaf(s2, p, C_1_3);
    p = fmaf(s2, p, 1.0f);
    float base = (float)(24 - e) * F_TWO_LN2;
    float rho2 = fmaf(-4.0f * s, p, base);
    return sqrtf(rho2);
}

void ngdbf_ref_sincos2pi(uint32_t i, float *c, float *s) {
    /* Quadrant q = i >> 22; the remainder r in [0, 2^22) is reflected to
     * r' = min(r, 2^22 - r) so that alpha = r' * 2pi 2^-24 is in [0, pi/4].
     * sin and cos of alpha from their Taylor series through alpha^9 and
     * alpha^10 (remainders below 3e-9). */
    uint32_t q = (i >> 22) & 3u;
    uint32_t r = i & 0x3FFFFFu;
    int reflect = r > 0x200000u;
    uint32_t rr = reflect ? (0x400000u - r) : r;
    float a = (float)rr * F_TWOPI_M24;
    float a2 = a * a;
    float ps = fmaf(a2, S_9, S_7);
    ps = fmaf(a2, ps, S_5);
    ps = fmaf(a2, ps, S_3);
    float sn = fmaf(a * a2, ps, a);
    float pc = fmaf(a2, K_10, K_8);
    pc = fmaf(a2, pc, K_6);
    pc = fmaf(a2, pc, K_4);
    pc = fmaf(a2, pc, K_2);
    float cs = fmaf(a2, pc, 1.0f);
    if (reflect) { float t = sn; sn = cs; cs = t; }
    /* rotate by q quarter turns */
    float co, si;
    switch (q) {
        case 0:  co = cs;  si = sn;  break;
        case 1:  co = -sn; si = cs;  break;
        case 2:  co = -cs; si = -sn; break;
        default: co = sn;  si = -cs; break;
    }
    *c = co;
    *s = si;
}

void ngdbf_ref_gauss_pair(uint32_t a, uint32_t b, float z[2]) {
    uint32_t m = (a >> 8) + 1u;
    uint32_t i = b >> 8;
    float rho = ngdbf_ref_rho(m);
    float c, s;
    ngdbf_ref_sincos2pi(i, &c, &s);
    z[0] = rho * c;
    z[1] = rho * s;
}

void ngdbf_ref_noise_quad(uint64_t seed, uint64_t frame, uint32_t t,
                          uint32_t quad, float z[4]) {
    /* counter = (bit quad, iteration, frame lo, frame hi); key = seed */
    uint32_t ctr[4] = {quad, t, (uint32_t)frame, (uint32_t)(frame >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    ngdbf_ref_philox4x32_10(ctr, key, r);
    ngdbf_ref_gauss_pair(r[0], r[1], &z[0]);
    ngdbf_ref_gauss_pair(r[2], r[3], &z[2]);
}

void ngdbf_ref_noise_block(uint64_t seed, uint64_t frame, uint32_t t,
                           uint32_t quad0, uint32_t n_quads, float *z) {
    for (uint32_t j = 0; j < n_quads; ++j)
        ngdbf_ref_noise_quad(seed, frame, t, quad0 + j, z + 4 * (size_t)j);
}

void ngdbf_ref_rho_range(uint32_t m0, uint32_t count, float *out) {
    for (uint32_t j = 0; j < count; ++j) out[j] = ngdbf_ref_rho(m0 + j);
}

void ngdbf_ref_sincos_range(uint32_t i0, uint32_t count, float *c, float *s) {
    for (uint32_t j = 0; j < count; ++j) ngdbf_ref_sincos2pi(i0 + j, &c[j], &s[j]);
}

/* ------------------------------------------------------------------ */
/* Code structure: N(i) from the CSR rows, M(k) built here as CSC.    */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n, m;
    const int32_t *row_ptr, *col_idx;   /* N(i) */
    int32_t *col_ptr, *row_idx;         /* M(k) */
} ref_code;

static int build_code(ref_code *h, int32_t n, int32_t m,
                      const int32_t *row_ptr, const int32_t *col_idx) {
    if (n <= 0 || m <= 0 || !row_ptr || !col_idx) return -1;
    int64_t nnz = row_ptr[m];
    if (row_ptr[0] != 0 || nnz < 0) return -1;
    for (int32_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return -1;
    for (int64_t e = 0; e < nnz; ++e)
        if (col_idx[e] < 0 || col_idx[e] >= n) return -1;
    h->n = n; h->m = m; h->row_ptr = row_ptr; h->col_idx = col_idx;
    h->col_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    h->row_idx = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    if (!h->col_ptr || !h->row_idx) return -1;
    for (int64_t e = 0; e < nnz; ++e) h->col_ptr[col_idx[e] + 1]++;
    for (int32_t k = 0; k < n; ++k) h->col_ptr[k + 1] += h->col_ptr[k];
    int32_t *fill = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!fill) return -1;
    memcpy(fill, h->col_ptr, (size_t)n * sizeof(int32_t));
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            h->row_idx[fill[col_idx[e]]++] = i;
    free(fill);
    return 0;
}

static void free_code(ref_code *h) {
    free(h->col_ptr);
    free(h->row_idx);
}

/* ------------------------------------------------------------------ */
/* FP32 decoder, one frame.                                           */
/* ------------------------------------------------------------------ */

typedef struct {
    const ref_code *h;
    const void *y;
    int32_t y_format;
    const float *sigma;
    float sigma_scalar;
    ngdbf_ref_params p;
    uint64_t seed, frame_base;
    uint8_t *out_bits;
    int32_t *out_iters;
    uint8_t *out_conv;
    uint8_t *trace;
    int64_t n_frames;
    int32_t n_threads;
    int use_f64;
} job;

static void pack_bits_from_x(const int *x, int32_t n, uint8_t *dst) {
    /* c_k = (1 - x_k)/2, bit k of byte k/8 (Sec. III-A bipolar map) */
    int32_t nb = (n + 7) / 8;
    memset(dst, 0, (size_t)nb);
    for (int32_t k = 0; k < n; ++k)
        if (x[k] < 0) dst[k >> 3] |= (uint8_t)(1u << (k & 7));
}

static float load_y(const job *J, int64_t f, int32_t k) {
    int32_t n = J->h->n;
    if (J->y_format == 1) {
        /* int8 storage: y = y_q / 16, exact in binary32 */
        int8_t q = ((const int8_t *)J->y)[f * n + k];
        return (float)q * 0.0625f;
    }
    return ((const float *)J->y)[f * n + k];
}

/* ------------------------------------------------------------------ */
/* Quantizer (Sec. IV-E) and threshold adaptation events (Sec. V-A).  */
/* ------------------------------------------------------------------ */

float ngdbf_ref_quant_half(float v, int32_t q_bits, float c) {
    /* g(v) = sign(v) (floor(|v| N_Q / 2Y_max) + 1/2) (2 Y_max / N_Q); the
     * levels stop at N_Q/2 - 1 on each side (zero is not a level).  Scaled
     * by N_Q / Y_max this is the odd integer sign(v) (2L + 1).  sign is the
     * signum, so g(0) = 0: a zero perturbation (eta = 0) adds nothing. */
    if (v == 0.0f) return 0.0f;
    float top = (float)((1 << q_bits) / 2 - 1);
    float L = floorf(fabsf(v) * c);
    if (L > top) L = top;                    /* NaN stays NaN               */
    float mag = 2.0f * L + 1.0f;
    return (v < 0.0f) ? -mag : mag;
}

static float quant_scale(int32_t q_bits, float ymax) {
    return (float)(1 << q_bits) / (2.0f * ymax);   /* fl32(N_Q / 2Y_max) */
}

int32_t ngdbf_ref_threshold_events(float theta, float lambda, float ymax,
                                   int32_t q_bits, int32_t t_max,
                                   double *values, int32_t *taus, int32_t cap) {
    float c = quant_scale(q_bits, ymax);
    float thr = theta;                       /* theta lambda^u, u = 0       */
    float prev = 0.0f;
    int32_t count = 0;
    for (int32_t u = 0; u <= t_max; ++u) {
        if (u > 0) thr = thr * lambda;
        float lev = ngdbf_ref_quant_half(thr, q_bits, c);
        if (u == 0 || lev != prev) {
            if (count < cap) {
                values[count] = (double)lev * (double)ymax / (double)(1 << q_bits);
                taus[count] = u;
            }
            ++count;
        }
        prev = lev;
    }
    return count;
}

/* ------------------------------------------------------------------ */
/* Shift-register noise reuse (Sec. V-B).                             */
/* ------------------------------------------------------------------ */

float ngdbf_ref_reuse_sample(uint64_t seed, uint64_t frame, int32_t n,
                             uint32_t t, int32_t k) {
    /* One new sample enters bit 0 each round and every register passes its
     * sample to the next bit: q_k(t) = q_{k-1}(t-1).  With the registers
     * preloaded from the stream r (bit k holds r[n-1-k] at t = 0), bit k
     * holds r[n-1+t-k] in round t. */
    uint32_t j = (uint32_t)(n - 1) + t - (uint32_t)k;
    float z4[4];
    ngdbf_ref_noise_quad(seed, frame, 0xFFFFFFFFu, j >> 2, z4);
    return z4[j & 3];
}

/* ------------------------------------------------------------------ */
/* Channel of Sec. III-A: y = c_hat + z, z ~ N(0, sigma^2).           */
/* ------------------------------------------------------------------ */

/* The synthetic channel: BPSK symbol c_hat_k = 1 - 2 c_k (all-zero codeword
 * when no codeword is given) plus sigma z_k, formed as fmaf(sigma, z_k,
 * c_hat_k), with z_k the standard-normal draw of bit k under the iteration
 * word 0xFFFFFFFE (a value no decoding round and not the noise-reuse stream
 * takes) for the frame's index, keyed by the channel's own seed.  int8
 * storage: y_q = clamp(rint(16 y), -127, 127), ties to even. */
int ngdbf_ref_channel(int32_t n, int64_t n_frames, const float *sigma,
                      float sigma_scalar, uint64_t seed, uint64_t frame_base,
                      const uint8_t *codewords, int32_t y_format, void *y) {
    if (n < 1 || n_frames < 0 || (y_format != 0 && y_format != 1)) return -1;
    if (n_frames > 0 && !y) return -1;
    int32_t nb = (n + 7) / 8;
    for (int64_t f = 0; f < n_frames; ++f) {
        float sg = sigma ? sigma[f] : sigma_scalar;
        uint64_t frame = frame_base + (uint64_t)f;
        for (int32_t k = 0; k < n; ++k) {
            float z4[4];
            ngdbf_ref_noise_quad(seed, frame, 0xFFFFFFFEu, (uint32_t)k >> 2, z4);
            int c = codewords ? (codewords[(size_t)f * nb + (k >> 3)] >> (k & 7)) & 1 : 0;
            float v = fmaf(sg, z4[k & 3], c ? -1.0f : 1.0f);
            if (y_format == 0) {
                ((float *)y)[(size_t)f * n + k] = v;
            } else {
                float q = rintf(16.0f * v);          /* 16 v is exact; rint: ties to even */
                if (!(q >= -127.0f)) q = -127.0f;    /* a NaN sample saturates low */
                if (q > 127.0f) q = 127.0f;
                ((int8_t *)y)[(size_t)f * n + k] = (int8_t)q;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Objective function (Sec. III-B) in exact fixed point.              */
/* ------------------------------------------------------------------ */

static int64_t fixed_sample(float v) {
    float a = v * 0x1p20f;                   /* exact unless it overflows   */
    if (!(a == a)) a = 0.0f;
    if (a > 0x1p40f) a = 0x1p40f;
    if (a < -0x1p40f) a = -0x1p40f;
    return (int64_t)rintf(a);                /* round half to even          */
}

static int64_t objective_fixed(const int *x, const float *yk, const int *s,
                               int32_t n, int32_t m) {
    int64_t F = 0;
    for (int32_t k = 0; k < n; ++k) F += (int64_t)x[k] * fixed_sample(yk[k]);
    for (int32_t i = 0; i < m; ++i) F += (int64_t)s[i] * ((int64_t)1 << 20);
    return F;
}

/* ------------------------------------------------------------------ */
/* FP32 / quantized decoder, one frame.                               */
/* ------------------------------------------------------------------ */

static void decode_frame_f32(const job *J, int64_t f, int *x, int *s,
                             float *yk, float *thr, int *X, int *flip, float *E) {
    const ref_code *h = J->h;
    const ngdbf_ref_params *p = &J->p;
    int32_t n = h->n, m = h->m, T = p->t_max, W = p->smooth_window;
    int32_t nb = (n + 7) / 8;
    uint64_t frame = J->frame_base + (uint64_t)f;
    float sigma = J->sigma ? J->sigma[f] : J->sigma_scalar;
    float qscale = p->eta * sigma;           /* std of q_k is eta*sigma   */
    uint8_t *trace = J->trace ? J->trace + (size_t)f * (size_t)T * nb : NULL;
    int Q = p->quant_bits;
    float qc = Q ? quant_scale(Q, p->ymax) : 0.0f;
    /* quantized weight w~ = g(w), in half-step units (Sec. IV-E) */
    float wq = Q ? ngdbf_ref_quant_half(p->w, Q, qc) : 0.0f;
    int mu = 1;                              /* mode switching (Sec. III-B) */
    int64_t f_prev = 0;

    /* Step 0 and x(0) = sign(y): saturate at Y_max, x_k = -1 iff y_k < 0 */
    for (int32_t k = 0; k < n; ++k) {
        float v = load_y(J, f, k);
        if (p->ymax > 0.0f) {
            if (v < -p->ymax) v = -p->ymax;
            if (v > p->ymax) v = p->ymax;
        }
        yk[k] = v;
        x[k] = (v < 0.0f) ? -1 : 1;
        thr[k] = p->theta;
        X[k] = 0;
    }

    for (int32_t t = 0;; ++t) {
        /* Step 1: s_i = prod_{j in N(i)} x_j */
        int unsatisfied = 0;
        for (int32_t i = 0; i < m; ++i) {
            int prod = 1;
            for (int32_t e = h->row_ptr[i]; e < h->row_ptr[i + 1]; ++e)
                prod *= x[h->col_idx[e]];
            s[i] = prod;
            if (prod < 0) unsatisfied = 1;
        }
        /* Sec. III-E: X_k accumulates x_k(t) over t = T-W .. T */
        if (W > 0 && t >= T - W)
            for (int32_t k = 0; k < n; ++k) X[k] += x[k];
        /* mode switching: mu drops to 0 for good once f(x(t)) < f(x(t-1)) */
        if (p->variant == 2) {
            int64_t fx = objective_fixed(x, yk, s, n, m);
            if (t > 0 && fx < f_prev) mu = 0;
            f_prev = fx;
        }
        if (!unsatisfied) {
            pack_bits_from_x(x, n, J->out_bits + (size_t)f * nb);
            J->out_iters[f] = t;
            if (J->out_conv) J->out_conv[f] = 1;
            return;
        }
        if (t == T) {
            if (W > 0)
                for (int32_t k = 0; k < n; ++k) x[k] = (X[k] < 0) ? -1 : 1;
            pack_bits_from_x(x, n, J->out_bits + (size_t)f * nb);
            J->out_iters[f] = T;
            if (J->out_conv) J->out_conv[f] = 0;
            return;
        }
        /* Step 2: E_k = x_k y_k + w sum_{i in M(k)} s_i + q_k.
         * Binary32: fmaf(qscale, z_k, fmaf(w, S_k, x_k*y_k)).
         * Quantized: x_k g(y_k) + g(w) S_k + g(qscale z_k) in half steps,
         * small integers, so the float sum is exact. */
        for (int32_t k = 0; k < n; ++k) {
            int S = 0;
            for (int32_t e = h->col_ptr[k]; e < h->col_ptr[k + 1]; ++e)
                S += s[h->row_idx[e]];
            float z;
            if (p->noise_reuse) {
                z = ngdbf_ref_reuse_sample(J->seed, frame, n, (uint32_t)t, k);
            } else {
                float z4[4];
                ngdbf_ref_noise_quad(J->seed, frame, (uint32_t)t, (uint32_t)k >> 2, z4);
                z = z4[k & 3];
            }
            if (Q) {
                float Y = ngdbf_ref_quant_half(yk[k], Q, qc);
                float qk = ngdbf_ref_quant_half(qscale * z, Q, qc);
                E[k] = (float)x[k] * Y + wq * (float)S + qk;
            } else {
                float xy = (float)x[k] * yk[k];
                float a = fmaf(p->w, (float)S, xy);
                E[k] = fmaf(qscale, z, a);
            }
        }
        /* Step 3 */
        int multi = (p->variant == 0) || (p->variant == 2 && mu == 1);
        if (multi) {
            /* 3b: flip iff E_k < theta_k (quantized: g(theta_k)) */
            for (int32_t k = 0; k < n; ++k) {
                float th = Q ? ngdbf_ref_quant_half(thr[k], Q, qc) : thr[k];
                flip[k] = E[k] < th;
            }
        } else {
            /* 3a: flip the single bit of least E_k; ties go to the lowest
             * index, NaN values are never chosen */
            int32_t best = -1;
            for (int32_t k = 0; k < n; ++k) {
                flip[k] = 0;
                if (E[k] == E[k] && (best < 0 || E[k] < E[best])) best = k;
            }
            if (best >= 0) flip[best] = 1;
        }
        /* all symbols update simultaneously from x(t) */
        for (int32_t k = 0; k < n; ++k) {
            if (flip[k]) {
                x[k] = -x[k];
                if (trace) trace[(size_t)t * nb + (k >> 3)] |= (uint8_t)(1u << (k & 7));
            } else if (multi) {
                thr[k] = thr[k] * p->lambda;     /* Sec. III-D, V-A */
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* FP64 decoder, one frame (statistical comparison).                  */
/* ------------------------------------------------------------------ */

static void noise_quad_f64(uint64_t seed, uint64_t frame, uint32_t t,
                           uint32_t quad, double z[4]) {
    uint32_t ctr[4] = {quad, t, (uint32_t)frame, (uint32_t)(frame >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    ngdbf_ref_philox4x32_10(ctr, key, r);
    for (int pr = 0; pr < 2; ++pr) {
        double u1 = (double)((r[2 * pr] >> 8) + 1u) * 0x1p-24;
        double phi = 2.0 * 3.14159265358979323846 * (double)(r[2 * pr + 1] >> 8) * 0x1p-24;
        double rho = sqrt(-2.0 * log(u1));
        z[2 * pr] = rho * cos(phi);
        z[2 * pr + 1] = rho * sin(phi);
    }
}

static void decode_frame_f64(const job *J, int64_t f, int *x, int *s,
                             double *yk, double *thr, int *X, int *flip) {
    const ref_code *h = J->h;
    const ngdbf_ref_params *p = &J->p;
    int32_t n = h->n, m = h->m, T = p->t_max, W = p->smooth_window;
    int32_t nb = (n + 7) / 8;
    uint64_t frame = J->frame_base + (uint64_t)f;
    double sigma = J->sigma ? J->sigma[f] : J->sigma_scalar;
    double qscale = (double)p->eta * sigma;
    for (int32_t k = 0; k < n; ++k) {
        double v = ((const float *)J->y)[f * n + k];
        if (p->ymax > 0.0f) {
            if (v < -(double)p->ymax) v = -(double)p->ymax;
            if (v > (double)p->ymax) v = (double)p->ymax;
        }
        yk[k] = v;
        x[k] = (v < 0.0) ? -1 : 1;
        thr[k] = p->theta;
        X[k] = 0;
    }
    for (int32_t t = 0;; ++t) {
        int unsatisfied = 0;
        for (int32_t i = 0; i < m; ++i) {
            int prod = 1;
            for (int32_t e = h->row_ptr[i]; e < h->row_ptr[i + 1]; ++e)
                prod *= x[h->col_idx[e]];
            s[i] = prod;
            if (prod < 0) unsatisfied = 1;
        }
        if (W > 0 && t >= T - W)
            for (int32_t k = 0; k < n; ++k) X[k] += x[k];
        if (!unsatisfied || t == T) {
            if (unsatisfied && W > 0)
                for (int32_t k = 0; k < n; ++k) x[k] = (X[k] < 0) ? -1 : 1;
            pack_bits_from_x(x, n, J->out_bits + (size_t)f * nb);
            J->out_iters[f] = t;
            if (J->out_conv) J->out_conv[f] = (uint8_t)!unsatisfied;
            return;
        }
        for (int32_t k = 0; k < n; ++k) {
            int S = 0;
            for (int32_t e = h->col_ptr[k]; e < h->col_ptr[k + 1]; ++e)
                S += s[h->row_idx[e]];
            double z4[4];
            noise_quad_f64(J->seed, frame, (uint32_t)t, (uint32_t)k >> 2, z4);
            double E = (double)x[k] * yk[k] + (double)p->w * S + qscale * z4[k & 3];
            flip[k] = E < thr[k];
        }
        for (int32_t k = 0; k < n; ++k) {
            if (flip[k]) x[k] = -x[k];
            else thr[k] = thr[k] * (double)p->lambda;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Frame loop over worker threads (frames are independent).           */
/* ------------------------------------------------------------------ */

typedef struct {
    const job *J;
    int32_t worker;
} worker_arg;

static void *worker_main(void *vp) {
    const worker_arg *wa = (const worker_arg *)vp;
    const job *J = wa->J;
    int32_t n = J->h->n, m = J->h->m;
    int *x = (int *)malloc((size_t)n * sizeof(int));
    int *s = (int *)malloc((size_t)m * sizeof(int));
    int *X = (int *)malloc((size_t)n * sizeof(int));
    int *flip = (int *)malloc((size_t)n * sizeof(int));
    double *yd = (double *)malloc((size_t)n * sizeof(double));
    double *td = (double *)malloc((size_t)n * sizeof(double));
    float *yf = (float *)malloc((size_t)n * sizeof(float));
    float *tf = (float *)malloc((size_t)n * sizeof(float));
    float *Ef = (float *)malloc((size_t)n * sizeof(float));
    if (x && s && X && flip && yd && td && yf && tf && Ef) {
        int32_t nt = J->n_threads > 1 ? J->n_threads : 1;
        for (int64_t f = wa->worker; f < J->n_frames; f += nt) {
            if (J->use_f64) decode_frame_f64(J, f, x, s, yd, td, X, flip);
            else decode_frame_f32(J, f, x, s, yf, tf, X, flip, Ef);
        }
    }
    free(x); free(s); free(X); free(flip); free(yd); free(td); free(yf); free(tf); free(Ef);
    return NULL;
}

static int run_job(job *J) {
    int32_t nt = J->n_threads > 1 ? J->n_threads : 1;
    if (J->n_frames > 0 && nt > J->n_frames) nt = (int32_t)J->n_frames;
    J->n_threads = nt;
    if (nt == 1) {
        worker_arg wa = {J, 0};
        worker_main(&wa);
        return 0;
    }
    pthread_t *th = (pthread_t *)malloc((size_t)nt * sizeof(pthread_t));
    worker_arg *wa = (worker_arg *)malloc((size_t)nt * sizeof(worker_arg));
    if (!th || !wa) { free(th); free(wa); return -1; }
    for (int32_t w = 0; w < nt; ++w) {
        wa[w].J = J;
        wa[w].worker = w;
        pthread_create(&th[w], NULL, worker_main, &wa[w]);
    }
    for (int32_t w = 0; w < nt; ++w) pthread_join(th[w], NULL);
    free(th);
    free(wa);
    return 0;
}

static int check_params(const ngdbf_ref_params *p) {
    if (!p) return -1;
    if (p->t_max < 0 || p->smooth_window < 0) return -1;
    if (p->variant < 0 || p->variant > 2) return -1;
    if (p->noise_reuse != 0 && p->noise_reuse != 1) return -1;
    if (p->quant_bits < 0 || p->quant_bits > 8) return -1;
    if (p->quant_bits && !(p->ymax > 0.0f)) return -1;   /* g needs Y_max  */
    if (p->quant_bits && p->variant == 2) return -1;     /* f is binary32  */
    return 0;
}

int ngdbf_ref_objective(int32_t n, int32_t m, const int32_t *row_ptr,
                        const int32_t *col_idx, const void *y, int32_t y_format,
                        int64_t n_frames, float ymax, const uint8_t *bits,
                        int64_t *out) {
    if (n_frames < 0 || (y_format != 0 && y_format != 1)) return -1;
    if (n_frames > 0 && (!y || !bits || !out)) return -1;
    ref_code h;
    memset(&h, 0, sizeof h);
    if (build_code(&h, n, m, row_ptr, col_idx)) { free_code(&h); return -1; }
    int *x = (int *)malloc((size_t)n * sizeof(int));
    int *s = (int *)malloc((size_t)m * sizeof(int));
    float *yk = (float *)malloc((size_t)n * sizeof(float));
    int rc = (x && s && yk) ? 0 : -1;
    ngdbf_ref_params p0;
    memset(&p0, 0, sizeof p0);
    job J = {&h, y, y_format, NULL, 0.0f, p0, 0, 0, NULL, NULL, NULL, NULL, n_frames, 1, 0};
    int32_t nb = (n + 7) / 8;
    for (int64_t f = 0; rc == 0 && f < n_frames; ++f) {
        for (int32_t k = 0; k < n; ++k) {
            float v = load_y(&J, f, k);
            if (ymax > 0.0f) {
                if (v < -ymax) v = -ymax;
                if (v > ymax) v = ymax;
            }
            yk[k] = v;
            x[k] = ((bits[(size_t)f * nb + (k >> 3)] >> (k & 7)) & 1u) ? -1 : 1;
        }
        for (int32_t i = 0; i < m; ++i) {
            int prod = 1;
            for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) prod *= x[col_idx[e]];
            s[i] = prod;
        }
        out[f] = objective_fixed(x, yk, s, n, m);
    }
    free(x); free(s); free(yk);
    free_code(&h);
    return rc;
}

int ngdbf_ref_decode(int32_t n, int32_t m, const int32_t *row_ptr,
                     const int32_t *col_idx, const void *y, int32_t y_format,
                     int64_t n_frames, const float *sigma, float sigma_scalar,
                     const ngdbf_ref_params *p, uint64_t seed,
                     uint64_t frame_base, uint8_t *out_bits,
                     int32_t *out_iters, uint8_t *out_conv, uint8_t *trace,
                     int32_t n_threads) {
    if (check_params(p) || n_frames < 0 || (y_format != 0 && y_format != 1))
        return -1;
    if (n_frames > 0 && (!y || !out_bits || !out_iters)) return -1;
    ref_code h;
    memset(&h, 0, sizeof h);
    if (build_code(&h, n, m, row_ptr, col_idx)) { free_code(&h); return -1; }
    if (trace)
        memset(trace, 0, (size_t)n_frames * (size_t)p->t_max * (size_t)((n + 7) / 8));
    job J = {&h, y, y_format, sigma, sigma_scalar, *p, seed, frame_base,
             out_bits, out_iters, out_conv, trace, n_frames, n_threads, 0};
    int rc = run_job(&J);
    free_code(&h);
    return rc;
}

int ngdbf_ref_decode_f64(int32_t n, int32_t m, const int32_t *row_ptr,
                         const int32_t *col_idx, const float *y,
                         int64_t n_frames, const float *sigma,
                         float sigma_scalar, const ngdbf_ref_params *p,
                         uint64_t seed, uint64_t frame_base,
                         uint8_t *out_bits, int32_t *out_iters,
                         uint8_t *out_conv, int32_t n_threads) {
    if (check_params(p) || n_frames < 0) return -1;
    /* the binary64 decoder covers the multi-bit binary32 algorithm only */
    if (p->variant || p->quant_bits || p->noise_reuse) return -1;
    if (n_frames > 0 && (!y || !out_bits || !out_iters)) return -1;
    ref_code h;
    memset(&h, 0, sizeof h);
    if (build_code(&h, n, m, row_ptr, col_idx)) { free_code(&h); return -1; }
    job J = {&h, y, 0, sigma, sigma_scalar, *p, seed, frame_base,
             out_bits, out_iters, out_conv, NULL, n_frames, n_threads, 1};
    int rc = run_job(&J);
    free_code(&h);
    return rc;
}
