/* Drives every entry point of the C oracle (oracle/sc_oracle.c) on small
 * random inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any out-of-bounds access, leak, overflow or
 * other undefined behaviour aborts with a report.  Prints "ok" at the end. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_encode(int log2n, const uint8_t* u, uint8_t* x);
int oracle_bhattacharyya(int log2n, double z0, double* lnz, double* ln1mz);
int64_t oracle_frozen_set(int log2n, double z0, int64_t n_frozen, double fer_bound, uint8_t* frozen, double* r_out);
int oracle_sc_decode(int log2n, int boxplus, const float* llr, const uint8_t* frozen, const uint8_t* fval,
                     const uint8_t* teacher, uint8_t* u_hat, void* leaf, uint8_t* beta_out);
int oracle_sc_decode_batch(int log2n, int boxplus, int n_frames, int shared_frozen, const float* llr,
                           const uint8_t* frozen, const uint8_t* fval, uint8_t* u_hat, int n_threads);
int oracle_phi_table(int frac, int len, int32_t* out);
int oracle_sc_decode_fixed(int log2n, int kind, const int32_t* llr, const uint8_t* frozen, const uint8_t* fval,
                           const uint8_t* teacher, uint8_t* u_hat, int32_t* leaf, const int32_t* table, int len);
int oracle_scl_decode(int log2n, int list, const float* llr, const uint8_t* frozen, const uint8_t* fval,
                      uint8_t* u_hat, float* pm_out);
int32_t oracle_f_fixed(int kind, int32_t a, int32_t b, const int32_t* table, int len);

static uint32_t rng = 12345u;
static uint32_t next(void) {
    rng ^= rng << 13;
    rng ^= rng >> 17;
    rng ^= rng << 5;
    return rng;
}

#define CHECK(x)                                                    \
    do {                                                            \
        if ((x) != 0) {                                             \
            fprintf(stderr, "failed: %s (line %d)\n", #x, __LINE__); \
            return 1;                                               \
        }                                                           \
    } while (0)

int main(void) {
    int32_t table[256];
    CHECK(oracle_phi_table(4, 256, table));
    for (int log2n = 0; log2n <= 11; ++log2n) {
        const int n = 1 << log2n;
        uint8_t* u = malloc((size_t)n);
        uint8_t* x = malloc((size_t)n);
        uint8_t* fr = malloc((size_t)n);
        uint8_t* fv = malloc((size_t)n);
        uint8_t* te = malloc((size_t)n);
        uint8_t* uh = malloc((size_t)n);
        uint8_t* be = malloc((size_t)n);
        float* llr = malloc(sizeof(float) * (size_t)n);
        float* lf = malloc(sizeof(float) * (size_t)n);
        double* ld = malloc(sizeof(double) * (size_t)n);
        double* lz = malloc(sizeof(double) * (size_t)n);
        double* lw = malloc(sizeof(double) * (size_t)n);
        int32_t* q = malloc(sizeof(int32_t) * (size_t)n);
        int32_t* ql = malloc(sizeof(int32_t) * (size_t)n);
        for (int i = 0; i < n; ++i) {
            u[i] = next() & 1;
            te[i] = next() & 1;
            llr[i] = ((int)(next() % 17) - 8) * 0.25f;
            q[i] = (int)(next() % 200) - 100;
        }
        CHECK(oracle_encode(log2n, u, x));
        CHECK(oracle_bhattacharyya(log2n, 0.3, lz, lw));
        if (oracle_frozen_set(log2n, 0.3, n / 3, 0.1, fr, lz) < 0) return 1;
        if (oracle_frozen_set(log2n, 0.3, -1, 0.1, fr, NULL) < 0) return 1;
        for (int i = 0; i < n; ++i) fv[i] = u[i] & fr[i];
        CHECK(oracle_sc_decode(log2n, 0, llr, fr, fv, NULL, uh, lf, be));
        CHECK(oracle_sc_decode(log2n, 0, llr, fr, fv, te, uh, NULL, NULL));
        CHECK(oracle_sc_decode(log2n, 1, llr, fr, fv, NULL, uh, ld, be));
        CHECK(oracle_sc_decode(log2n, 1, llr, fr, fv, te, uh, NULL, NULL));
        CHECK(oracle_sc_decode_fixed(log2n, 0, q, fr, fv, NULL, uh, ql, table, 256));
        CHECK(oracle_sc_decode_fixed(log2n, 1, q, fr, fv, te, uh, NULL, table, 256));
        for (int list = 1; list <= 8; list *= 2) {
            float pm = 0.0f;
            CHECK(oracle_scl_decode(log2n, list, llr, fr, fv, uh, &pm));
        }
        if (log2n >= 1) {
            const int frames = 5;
            float* bl = malloc(sizeof(float) * (size_t)n * frames);
            uint8_t* bf = malloc((size_t)n * frames);
            uint8_t* bv = malloc((size_t)n * frames);
            uint8_t* bu = malloc((size_t)n * frames);
            for (int k = 0; k < frames; ++k) {
                memcpy(bl + (size_t)k * n, llr, sizeof(float) * (size_t)n);
                memcpy(bf + (size_t)k * n, fr, (size_t)n);
                memcpy(bv + (size_t)k * n, fv, (size_t)n);
            }
            CHECK(oracle_sc_decode_batch(log2n, log2n & 1, frames, 0, bl, bf, bv, bu, 3));
            CHECK(oracle_sc_decode_batch(log2n, 0, frames, 1, bl, fr, bv, bu, 2));
            free(bl);
            free(bf);
            free(bv);
            free(bu);
        }
        free(u);
        free(x);
        free(fr);
        free(fv);
        free(te);
        free(uh);
        free(be);
        free(llr);
        free(lf);
        free(ld);
        free(lz);
        free(lw);
        free(q);
        free(ql);
    }
    for (int a = -40000; a <= 40000; a += 997)
        for (int b = -300; b <= 300; b += 37) (void)oracle_f_fixed(1, a, b, table, 256);
    printf("ok\n");
    return 0;
}
