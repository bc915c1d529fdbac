/* Drives every decoder of the oracle on small inputs; built with
 * -fsanitize=address,undefined by tests/test_oracle_sanitize.py so that any
 * out-of-bounds access, leak or undefined behaviour in the oracle fails. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/ngdbf_oracle.h"

/* a (3,6) code with n = 24 built from a cyclic pattern */
static void make_code(int32_t *row_ptr, int32_t *col_idx) {
    for (int i = 0; i <= 12; ++i) row_ptr[i] = 6 * i;
    for (int i = 0; i < 12; ++i)
        for (int e = 0; e < 6; ++e) col_idx[6 * i + e] = (2 * i + 5 * e + (e > 2 ? 1 : 0)) % 24;
    /* sort and de-duplicate by construction: shift repeats */
    for (int i = 0; i < 12; ++i) {
        int32_t *r = col_idx + 6 * i;
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < a; ++b)
                while (r[a] == r[b]) { r[a] = (r[a] + 1) % 24; b = -1; break; }
    }
}

int main(void) {
    int32_t row_ptr[13], col_idx[72];
    make_code(row_ptr, col_idx);
    const int F = 40, n = 24;
    float *y = malloc(sizeof(float) * F * n);
    int8_t *y8 = malloc((size_t)F * n);
    float *sig = malloc(sizeof(float) * F);
    unsigned s = 12345;
    for (int i = 0; i < F * n; ++i) {
        s = s * 1103515245u + 12345u;
        y[i] = 1.0f + ((float)(s >> 9) / 8388608.0f - 0.5f) * 2.4f;
        y8[i] = (int8_t)(y[i] * 16.0f);
    }
    for (int f = 0; f < F; ++f) sig[f] = 0.5f + 0.01f * (float)f;
    uint8_t *bits = malloc((size_t)F * 3), *conv = malloc((size_t)F);
    int32_t *iters = malloc(sizeof(int32_t) * F);
    int64_t *obj = malloc(sizeof(int64_t) * F);
    const int T = 30;
    uint8_t *trace = malloc((size_t)F * T * 3);
    int fails = 0;
    for (int variant = 0; variant <= 2; ++variant)
        for (int q = 0; q <= 5; q += 5)
            for (int reuse = 0; reuse <= 1; ++reuse) {
                if (q && variant == 2) continue;
                ngdbf_ref_params p = {0.75f, -0.7f, 0.98f, 0.9f, 1.75f, T, 8, variant, q, reuse};
                for (int fmt = 0; fmt <= 1; ++fmt) {
                    int rc = ngdbf_ref_decode(n, 12, row_ptr, col_idx, fmt ? (const void *)y8 : (const void *)y,
                                              fmt, F, sig, 0.0f, &p, 7, 3, bits, iters, conv, trace, 3);
                    if (rc) { fprintf(stderr, "decode rc %d (v%d q%d r%d)\n", rc, variant, q, reuse); ++fails; }
                }
            }
    ngdbf_ref_params p64 = {0.75f, -0.7f, 0.98f, 0.9f, 2.5f, T, 8, 0, 0, 0};
    if (ngdbf_ref_decode_f64(n, 12, row_ptr, col_idx, y, F, NULL, 0.6f, &p64, 7, 0, bits, iters, conv, 2))
        ++fails;
    if (ngdbf_ref_objective(n, 12, row_ptr, col_idx, y, 0, F, 2.5f, bits, obj)) ++fails;
    double vals[16];
    int32_t taus[16];
    if (ngdbf_ref_threshold_events(-0.9f, 0.99f, 2.5f, 5, 300, vals, taus, 16) != 6) ++fails;
    float z[8];
    ngdbf_ref_noise_block(1, 2, 3, 0, 2, z);
    (void)ngdbf_ref_reuse_sample(1, 2, n, 5, 3);
    free(y); free(y8); free(sig); free(bits); free(conv); free(iters); free(obj); free(trace);
    printf(fails ? "FAILED\n" : "ok\n");
    return fails ? 1 : 0;
}
