/*
 * Plain CPU oracle for successive-cancellation (SC) decoding of polar codes.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU library, and the product path never
 * links or calls it.
 *
 * What it follows (Jouguet & Kunz-Jacques, "High performance error correction
 * for quantum key distribution using polar codes"):
 *   - Section 1: the encoding step is skipped in QKD; the message equals the
 *     string sent and the frozen ("parity") values are revealed, so the decoder
 *     is given the channel LLRs of Bob's string and the frozen values.
 *   - Section 3: channel polarisation (Arikan's construction, cited there as
 *     [Ari08]); the lowest-capacity synthetic channels are frozen, and the
 *     frozen set can be chosen so that a union bound on the frame error rate
 *     stays below 0.1.
 *   - Section 4: a recursive SC decoder, O(N log N), whose LLR updates are the
 *     exact check-node update written with phi(x) = log tanh(x/2); the
 *     min-sum update is the usual approximation of that same function.
 *
 * Bits are one byte each (0/1) so every step reads like the definition.
 * Compile with -O2 -ffp-contract=off -fno-fast-math: no FMA contraction, no
 * reassociation, denormals preserved.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Encoder: x = u * G_N over GF(2), G_N = F^{(x)n}, F = [[1,0],[1,1]],       */
/* natural index order (no bit-reversal permutation).                      */
/* Written as the half recursion x = [(u_a ^ u_b) G_{N/2}, u_b G_{N/2}],     */
/* which is the Kronecker structure of G_N (Section 3, [Ari08]).            */
/* ------------------------------------------------------------------------ */
static void encode_rec(const uint8_t* u, uint8_t* x, int64_t n) {
    if (n == 1) {
        x[0] = u[0];
        return;
    }
    int64_t h = n / 2;
    uint8_t* a = (uint8_t*)malloc((size_t)h);
    for (int64_t j = 0; j < h; ++j) a[j] = (uint8_t)(u[j] ^ u[j + h]);
    encode_rec(a, x, h);          /* first half: (u_a ^ u_b) G_{N/2} */
    encode_rec(u + h, x + h, h);  /* second half: u_b G_{N/2}        */
    free(a);
}

int oracle_encode(int log2n, const uint8_t* u, uint8_t* x) {
    if (log2n < 0 || log2n > 30 || !u || !x) return -1;
    int64_t n = (int64_t)1 << log2n;
    uint8_t* tmp = (uint8_t*)malloc((size_t)n);
    encode_rec(u, tmp, n);
    memcpy(x, tmp, (size_t)n);
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bhattacharyya parameters of the synthetic channels (Section 3).          */
/* One polarisation step maps Z to Z- = 2Z - Z^2 (the "minus", worse        */
/* channel, decoded first) and Z+ = Z^2 (the "plus" channel).  Index i with */
/* bits b_{n-1}..b_0 applies the step chosen by b_{n-1} first.              */
/* To avoid saturation of Z at 1.0 in double, the pair (ln Z, ln(1-Z)) is   */
/* carried:                                                                 */
/*   minus: ln(1-Z') = 2 ln(1-Z);  ln Z' = ln Z + log1p(1-Z)  (Z < 1/2)     */
/*                                        = log1mexp(2 ln(1-Z)) (otherwise) */
/*   plus:  ln Z'    = 2 ln Z;     ln(1-Z') = ln(1-Z) + log1p(Z) (Z > 1/2)  */
/*                                        = log1mexp(2 ln Z)   (otherwise)  */
/* log1mexp(x) = ln(1 - e^x) for x < 0, two-branch form (Maechler 2012).    */
/* ------------------------------------------------------------------------ */
static double log1mexp(double x) {
    if (x > -0.6931471805599453) return log(-expm1(x));
    return log1p(-exp(x));
}

int oracle_bhattacharyya(int log2n, double z0, double* lnz, double* ln1mz) {
    if (log2n < 0 || log2n > 30 || !(z0 > 0.0) || !(z0 < 1.0) || !lnz || !ln1mz) return -1;
    int64_t n = (int64_t)1 << log2n;
    double* az = (double*)malloc(sizeof(double) * (size_t)n);
    double* aw = (double*)malloc(sizeof(double) * (size_t)n);
    double* bz = (double*)malloc(sizeof(double) * (size_t)n);
    double* bw = (double*)malloc(sizeof(double) * (size_t)n);
    az[0] = log(z0);
    aw[0] = log1p(-z0);
    int64_t cnt = 1;
    for (int lev = 0; lev < log2n; ++lev) {
        for (int64_t j = 0; j < cnt; ++j) {
            double lz = az[j], lw = aw[j];
            double z = exp(lz);
            /* minus child at 2j */
            double mw = 2.0 * lw;
            double mz = (z < 0.5) ? lz + log1p(exp(lw)) : log1mexp(mw);
            /* plus child at 2j+1 */
            double pz = 2.0 * lz;
            double pw = (z > 0.5) ? lw + log1p(exp(lz)) : log1mexp(pz);
            bz[2 * j] = mz;
            bw[2 * j] = mw;
            bz[2 * j + 1] = pz;
            bw[2 * j + 1] = pw;
        }
        cnt *= 2;
        double* t;
        t = az; az = bz; bz = t;
        t = aw; aw = bw; bw = t;
    }
    memcpy(lnz, az, sizeof(double) * (size_t)n);
    memcpy(ln1mz, aw, sizeof(double) * (size_t)n);
    free(az); free(aw); free(bz); free(bw);
    return 0;
}

/* Frozen set: the n_frozen synthetic channels with the smallest reliability
 * r_i = ln((1-Z_i)/Z_i) are frozen (Section 3: lowest-capacity bits are
 * revealed).  Exact ties freeze the lower index first. */
typedef struct { double r; int64_t i; } rank_t;

static int cmp_rank(const void* pa, const void* pb) {
    const rank_t* a = (const rank_t*)pa;
    const rank_t* b = (const rank_t*)pb;
    if (a->r < b->r) return -1;
    if (a->r > b->r) return 1;
    return (a->i < b->i) ? -1 : (a->i > b->i);
}

/* n_frozen >= 0: freeze that many.  n_frozen < 0: union-bound rule, i.e.
 * K = the largest k such that the sum of the k smallest Z_i is <= fer_bound
 * (Section 3: the frozen set is chosen so that a bound on the FER is 0.1),
 * and N - K channels are frozen.  Returns the number frozen, or -1. */
int64_t oracle_frozen_set(int log2n, double z0, int64_t n_frozen, double fer_bound,
                          uint8_t* frozen, double* r_out) {
    if (log2n < 0 || log2n > 30 || !frozen) return -1;
    int64_t n = (int64_t)1 << log2n;
    if (n_frozen > n) return -1;
    double* lz = (double*)malloc(sizeof(double) * (size_t)n);
    double* lw = (double*)malloc(sizeof(double) * (size_t)n);
    if (oracle_bhattacharyya(log2n, z0, lz, lw) != 0) { free(lz); free(lw); return -1; }
    rank_t* rk = (rank_t*)malloc(sizeof(rank_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        rk[i].r = lw[i] - lz[i];
        rk[i].i = i;
        if (r_out) r_out[i] = rk[i].r;
    }
    qsort(rk, (size_t)n, sizeof(rank_t), cmp_rank);
    if (n_frozen < 0) {
        /* best channels are at the end of the ascending-r order */
        double sum = 0.0;
        int64_t k = 0;
        while (k < n) {
            double z = exp(lz[rk[n - 1 - k].i]);
            if (sum + z > fer_bound) break;
            sum += z;
            ++k;
        }
        n_frozen = n - k;
    }
    memset(frozen, 0, (size_t)n);
    for (int64_t t = 0; t < n_frozen; ++t) frozen[rk[t].i] = 1;
    free(rk); free(lz); free(lw);
    return n_frozen;
}

/* ------------------------------------------------------------------------ */
/* SC decoding (Section 4: recursive decoder; [Ari08]).                      */
/*                                                                          */
/* dec(alpha[0..M)):                                                        */
/*   M == 1: u = frozen value if frozen, else [alpha < 0]                   */
/*   else:   alpha_L[j] = f(alpha[j], alpha[j+M/2]);      beta_L = dec(L)   */
/*           alpha_R[j] = alpha[j+M/2] + (1-2 beta_L[j]) alpha[j]           */
/*                                                         beta_R = dec(R)  */
/*           return [beta_L ^ beta_R, beta_R]                               */
/* Leaves are reached in index order, so u-hat comes out in natural order.  */
/*                                                                          */
/* Teacher forcing: when a teacher vector is given, the partial sums use    */
/* the teacher's bits instead of this decoder's own decisions, so leaf LLRs */
/* can be compared past a decision that differs.                            */
/* ------------------------------------------------------------------------ */

/* Min-sum check update in FP32: sign(a) sign(b) min(|a|,|b|), the sign taken
 * from the IEEE sign bits. */
static float f_minsum(float a, float b) {
    float m = fminf(fabsf(a), fabsf(b));
    return (signbit(a) != signbit(b)) ? -m : m;
}

/* Variable update g = b + (1 - 2u) a; multiplying by +-1 is exact, so this is
 * one FP32 addition. */
static float g_f32(float a, float b, int u) { return u ? b - a : b + a; }

/* Exact check update, box-plus 2 atanh(tanh(a/2) tanh(b/2)), in FP64.
 * If min(|a|,|b|) <= 1 the tanh form is used (its product stays <= tanh(1/2),
 * so atanh never saturates); otherwise the equivalent log form
 * s (m + log1p(e^-(A+B)) - log1p(e^-|A-B|)) is used, whose result is at least
 * 1 - ln 2, so it cannot cancel badly. */
static double f_boxplus(double a, double b) {
    double A = fabs(a), B = fabs(b);
    double m = fmin(A, B);
    double s = (signbit(a) != signbit(b)) ? -1.0 : 1.0;
    if (m <= 1.0) return s * 2.0 * atanh(tanh(A / 2.0) * tanh(B / 2.0));
    return s * (m + log1p(exp(-(A + B))) - log1p(exp(-fabs(A - B))));
}

static double g_f64(double a, double b, int u) { return u ? b - a : b + a; }

typedef struct {
    const uint8_t* frozen;
    const uint8_t* fval;
    const uint8_t* teacher;
    uint8_t* u_hat;
    void* leaf;          /* float* (min-sum) or double* (box-plus), nullable */
    int boxplus;
    void** alpha_lvl;    /* per depth: child LLR buffer of size N >> (d+1) */
    uint8_t** bl_lvl;    /* per depth: beta of the left child  */
    uint8_t** br_lvl;    /* per depth: beta of the right child */
} sc_ctx;

static void dec_minsum(const float* alpha, int64_t m, int64_t off, int depth, sc_ctx* c,
                       uint8_t* beta) {
    if (m == 1) {
        float L = alpha[0];
        if (c->leaf) ((float*)c->leaf)[off] = L;
        int u = c->frozen[off] ? c->fval[off] : (L < 0.0f);
        c->u_hat[off] = (uint8_t)u;
        beta[0] = c->teacher ? c->teacher[off] : (uint8_t)u;
        return;
    }
    int64_t h = m / 2;
    float* a = (float*)c->alpha_lvl[depth];
    uint8_t* bl = c->bl_lvl[depth];
    uint8_t* br = c->br_lvl[depth];
    for (int64_t j = 0; j < h; ++j) a[j] = f_minsum(alpha[j], alpha[j + h]);
    dec_minsum(a, h, off, depth + 1, c, bl);
    for (int64_t j = 0; j < h; ++j) a[j] = g_f32(alpha[j], alpha[j + h], bl[j]);
    dec_minsum(a, h, off + h, depth + 1, c, br);
    for (int64_t j = 0; j < h; ++j) {
        beta[j] = (uint8_t)(bl[j] ^ br[j]);
        beta[j + h] = br[j];
    }
}

static void dec_boxplus(const double* alpha, int64_t m, int64_t off, int depth, sc_ctx* c,
                        uint8_t* beta) {
    if (m == 1) {
        double L = alpha[0];
        if (c->leaf) ((double*)c->leaf)[off] = L;
        int u = c->frozen[off] ? c->fval[off] : (L < 0.0);
        c->u_hat[off] = (uint8_t)u;
        beta[0] = c->teacher ? c->teacher[off] : (uint8_t)u;
        return;
    }
    int64_t h = m / 2;
    double* a = (double*)c->alpha_lvl[depth];
    uint8_t* bl = c->bl_lvl[depth];
    uint8_t* br = c->br_lvl[depth];
    for (int64_t j = 0; j < h; ++j) a[j] = f_boxplus(alpha[j], alpha[j + h]);
    dec_boxplus(a, h, off, depth + 1, c, bl);
    for (int64_t j = 0; j < h; ++j) a[j] = g_f64(alpha[j], alpha[j + h], bl[j]);
    dec_boxplus(a, h, off + h, depth + 1, c, br);
    for (int64_t j = 0; j < h; ++j) {
        beta[j] = (uint8_t)(bl[j] ^ br[j]);
        beta[j + h] = br[j];
    }
}

/* Decode one frame.  boxplus = 0: FP32 min-sum, leaf is float[N].
 * boxplus = 1: FP64 exact box-plus from the FP32 channel LLRs, leaf is
 * double[N].  teacher and leaf may be NULL.  beta_out (nullable) receives the
 * root partial sums, i.e. x-hat = u-hat G_N.  Returns 0 or -1. */
int oracle_sc_decode(int log2n, int boxplus, const float* llr, const uint8_t* frozen,
                     const uint8_t* fval, const uint8_t* teacher, uint8_t* u_hat, void* leaf,
                     uint8_t* beta_out) {
    if (log2n < 0 || log2n > 30 || !llr || !frozen || !fval || !u_hat) return -1;
    int64_t n = (int64_t)1 << log2n;
    size_t esz = boxplus ? sizeof(double) : sizeof(float);
    sc_ctx c;
    c.frozen = frozen;
    c.fval = fval;
    c.teacher = teacher;
    c.u_hat = u_hat;
    c.leaf = leaf;
    c.boxplus = boxplus;
    c.alpha_lvl = (void**)calloc((size_t)log2n + 1, sizeof(void*));
    c.bl_lvl = (uint8_t**)calloc((size_t)log2n + 1, sizeof(uint8_t*));
    c.br_lvl = (uint8_t**)calloc((size_t)log2n + 1, sizeof(uint8_t*));
    for (int d = 0; d < log2n; ++d) {
        int64_t h = n >> (d + 1);
        c.alpha_lvl[d] = malloc(esz * (size_t)h);
        c.bl_lvl[d] = (uint8_t*)malloc((size_t)h);
        c.br_lvl[d] = (uint8_t*)malloc((size_t)h);
    }
    uint8_t* beta = (uint8_t*)malloc((size_t)n);
    if (boxplus) {
        double* root = (double*)malloc(sizeof(double) * (size_t)n);
        for (int64_t j = 0; j < n; ++j) root[j] = (double)llr[j];
        dec_boxplus(root, n, 0, 0, &c, beta);
        free(root);
    } else {
        dec_minsum(llr, n, 0, 0, &c, beta);
    }
    if (beta_out) memcpy(beta_out, beta, (size_t)n);
    free(beta);
    for (int d = 0; d < log2n; ++d) {
        free(c.alpha_lvl[d]);
        free(c.bl_lvl[d]);
        free(c.br_lvl[d]);
    }
    free(c.alpha_lvl);
    free(c.bl_lvl);
    free(c.br_lvl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fixed-point SC (Section 4: the decoder keeps LLRs in fixed point, and its */
/* check update uses phi(x) = -ln tanh(x/2) from a table, the paper's main   */
/* optimization; phi is its own inverse, so the exact update is             */
/* f = sign(a) sign(b) phi(phi(|a|) + phi(|b|))).                           */
/*                                                                          */
/* LLRs are integers in units of 2^-FRAC (FRAC = 4 here), saturated to      */
/* +-32767 (int16 range), or for kind 2 to +-127 (int8 range, in whatever   */
/* units: min-sum is the same at every scale but for the saturation).       */
/* Check updates:                                                           */
/*   kind 0, saturating min-sum: f = sign(a) sign(b) min(|a|, |b|)           */
/*   kind 1, phi table:          f = sign(a) sign(b) min(T[min(T[|a|] +     */
/*       T[|b|], len-1)], |a|, |b|), T[i] = phi(i 2^-FRAC) in the same units */
/*       (T[i] = 0 beyond the table), the min with |a|, |b| because the     */
/*       exact update never exceeds either magnitude (it also stands in for  */
/*       T[0] = phi(0) = infinity)                                           */
/*   kind 2, saturating min-sum on 8-bit integers: f as kind 0               */
/* Variable update for all: g = sat(b + (1 - 2u) a).  Decisions [L < 0].     */
/* ------------------------------------------------------------------------ */
#define FIXED_MAX 32767
#define FIXED8_MAX 127

static int32_t sat_to(int32_t x, int32_t lim) { return x > lim ? lim : (x < -lim ? -lim : x); }

/* T[i] = round(phi(i 2^-frac) 2^frac), phi(x) = ln(1 + 2 / expm1(x)) (the
 * same function as -ln tanh(x/2), without cancellation for large x),
 * rounded half up, capped at FIXED_MAX; T[0] = FIXED_MAX. */
int oracle_phi_table(int frac, int len, int32_t* out) {
    if (frac < 0 || frac > 12 || len < 2 || !out) return -1;
    const double step = ldexp(1.0, -frac);
    out[0] = FIXED_MAX;
    for (int i = 1; i < len; ++i) {
        double v = log1p(2.0 / expm1(i * step)) / step;
        double r = floor(v + 0.5);
        out[i] = r > FIXED_MAX ? FIXED_MAX : (int32_t)r;
    }
    return 0;
}

typedef struct {
    const uint8_t* frozen;
    const uint8_t* fval;
    const uint8_t* teacher;
    uint8_t* u_hat;
    int32_t* leaf;
    int kind;
    int32_t max;  /* saturation: FIXED_MAX, or FIXED8_MAX for kind 2 */
    const int32_t* table;
    int len;
    int32_t** alpha_lvl;
    uint8_t** bl_lvl;
    uint8_t** br_lvl;
} fx_ctx;

static int32_t fx_phi(const fx_ctx* c, int32_t x) { return x < c->len ? c->table[x] : 0; }

static int32_t fx_f(const fx_ctx* c, int32_t a, int32_t b) {
    int32_t A = a < 0 ? -a : a, B = b < 0 ? -b : b;
    int32_t m = A < B ? A : B;
    int32_t r = m;
    if (c->kind == 1) {
        int32_t s = fx_phi(c, A) + fx_phi(c, B);
        int32_t t = fx_phi(c, s < c->len ? s : c->len - 1);
        r = t < m ? t : m;
    }
    return ((a < 0) != (b < 0)) ? -r : r;
}

static int32_t fx_g(const fx_ctx* c, int32_t a, int32_t b, int u) { return sat_to(u ? b - a : b + a, c->max); }

static void dec_fixed(const int32_t* alpha, int64_t m, int64_t off, int depth, fx_ctx* c, uint8_t* beta) {
    if (m == 1) {
        int32_t L = alpha[0];
        if (c->leaf) c->leaf[off] = L;
        int u = c->frozen[off] ? c->fval[off] : (L < 0);
        c->u_hat[off] = (uint8_t)u;
        beta[0] = c->teacher ? c->teacher[off] : (uint8_t)u;
        return;
    }
    int64_t h = m / 2;
    int32_t* a = c->alpha_lvl[depth];
    uint8_t* bl = c->bl_lvl[depth];
    uint8_t* br = c->br_lvl[depth];
    for (int64_t j = 0; j < h; ++j) a[j] = fx_f(c, alpha[j], alpha[j + h]);
    dec_fixed(a, h, off, depth + 1, c, bl);
    for (int64_t j = 0; j < h; ++j) a[j] = fx_g(c, alpha[j], alpha[j + h], bl[j]);
    dec_fixed(a, h, off + h, depth + 1, c, br);
    for (int64_t j = 0; j < h; ++j) {
        beta[j] = (uint8_t)(bl[j] ^ br[j]);
        beta[j + h] = br[j];
    }
}

/* Decode one frame in fixed point.  llr: N integers (channel LLRs in units
 * of 2^-frac, inside +-32767, or +-127 for kind 2); kind 0 saturating
 * min-sum, 1 phi table (table of len entries, from oracle_phi_table), 2
 * saturating min-sum on 8-bit integers; leaf (nullable) receives the N
 * decision LLRs.  Returns 0 or -1. */
int oracle_sc_decode_fixed(int log2n, int kind, const int32_t* llr, const uint8_t* frozen, const uint8_t* fval,
                           const uint8_t* teacher, uint8_t* u_hat, int32_t* leaf, const int32_t* table,
                           int len) {
    if (log2n < 0 || log2n > 30 || !llr || !frozen || !fval || !u_hat) return -1;
    if (kind != 0 && kind != 1 && kind != 2) return -1;
    if (kind == 1 && (!table || len < 2)) return -1;
    const int32_t lim = kind == 2 ? FIXED8_MAX : FIXED_MAX;
    int64_t n = (int64_t)1 << log2n;
    for (int64_t j = 0; j < n; ++j)
        if (llr[j] > lim || llr[j] < -lim) return -1;
    fx_ctx c;
    c.frozen = frozen;
    c.fval = fval;
    c.teacher = teacher;
    c.u_hat = u_hat;
    c.leaf = leaf;
    c.kind = kind;
    c.max = lim;
    c.table = table;
    c.len = len;
    c.alpha_lvl = (int32_t**)calloc((size_t)log2n + 1, sizeof(int32_t*));
    c.bl_lvl = (uint8_t**)calloc((size_t)log2n + 1, sizeof(uint8_t*));
    c.br_lvl = (uint8_t**)calloc((size_t)log2n + 1, sizeof(uint8_t*));
    for (int d = 0; d < log2n; ++d) {
        int64_t h = n >> (d + 1);
        c.alpha_lvl[d] = (int32_t*)malloc(sizeof(int32_t) * (size_t)h);
        c.bl_lvl[d] = (uint8_t*)malloc((size_t)h);
        c.br_lvl[d] = (uint8_t*)malloc((size_t)h);
    }
    uint8_t* beta = (uint8_t*)malloc((size_t)n);
    dec_fixed(llr, n, 0, 0, &c, beta);
    free(beta);
    for (int d = 0; d < log2n; ++d) {
        free(c.alpha_lvl[d]);
        free(c.bl_lvl[d]);
        free(c.br_lvl[d]);
    }
    free(c.alpha_lvl);
    free(c.bl_lvl);
    free(c.br_lvl);
    return 0;
}

/* Scalar updates exported for the tests that pin them. */
/* ------------------------------------------------------------------------ */
/* SC list decoding (the list decoders the paper names as an improvement of */
/* SC in Section 4; Tal and Vardy, with the LLR form of the path metric of  */
/* Balatsoukas-Stimming, Bastani Parizi and Burg).  FP32 min-sum f and g as */
/* in oracle_sc_decode.  Up to L paths are kept; each carries its decided   */
/* bits and a path metric PM (FP32, starts at 0).  At leaf i every path     */
/* computes its leaf LLR lambda by SC on its own decisions, and:            */
/*   frozen i:  u = frozen value, PM += |lambda| if u != [lambda < 0]        */
/*   info i:    each path p offers (u = b, PM_p + (b != [lambda < 0] ?       */
/*              |lambda| : 0)) for b = 0, 1; the candidates are ordered by   */
/*              (metric, p, b) and the first min(L, count) become the new    */
/*              paths, in that order                                         */
/* The output is the path of least PM, ties to the lower path index; its    */
/* metric goes to *pm_out.                                                   */
/* Per path the state is the LLRs of the current node at every depth and    */
/* the decided bits; the partial sums a g needs are the left sibling's      */
/* decisions re-encoded.  A surviving candidate copies its parent's state.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    float* a;    /* depth d (1..n) at a + (N - (N >> (d - 1))), N >> d floats */
    uint8_t* u;  /* decided bits 0 .. i-1 */
    float pm;
} scl_path;

static float* scl_level(const scl_path* p, int64_t n, int d) { return p->a + (n - (n >> (d - 1))); }

/* LLR of leaf i for one path: the nodes that change between leaves i-1 and  */
/* i are recomputed, from depth n - t (t = trailing zeros of i) down.        */
static float scl_leaf(scl_path* p, const float* llr, int log2n, int64_t i, uint8_t* beta) {
    const int64_t n = (int64_t)1 << log2n;
    int top = 1;
    if (i > 0) {
        int t = 0;
        while (((i >> t) & 1) == 0) ++t;
        top = log2n - t; /* depth of the new right child */
        const int64_t m = n >> (top - 1), h = m / 2; /* parent size */
        const float* par = top == 1 ? llr : scl_level(p, n, top - 1);
        float* out = scl_level(p, n, top);
        /* left sibling: leaves [i - h, i), re-encoded */
        encode_rec(p->u + (i - h), beta, h);
        for (int64_t j = 0; j < h; ++j) out[j] = g_f32(par[j], par[j + h], beta[j]);
        ++top;
    }
    for (int d = top; d <= log2n; ++d) {
        const int64_t m = n >> (d - 1), h = m / 2;
        const float* par = d == 1 ? llr : scl_level(p, n, d - 1);
        float* out = scl_level(p, n, d);
        for (int64_t j = 0; j < h; ++j) out[j] = f_minsum(par[j], par[j + h]);
    }
    return log2n == 0 ? llr[0] : scl_level(p, n, log2n)[0];
}

typedef struct {
    float pm;
    int parent, bit;
} scl_cand;

static int scl_before(const scl_cand* x, const scl_cand* y) {
    if (x->pm != y->pm) return x->pm < y->pm;
    if (x->parent != y->parent) return x->parent < y->parent;
    return x->bit < y->bit;
}

int oracle_scl_decode(int log2n, int list, const float* llr, const uint8_t* frozen, const uint8_t* fval,
                      uint8_t* u_hat, float* pm_out) {
    if (log2n < 0 || log2n > 20 || list < 1 || list > 64 || !llr || !frozen || !fval || !u_hat) return -1;
    const int64_t n = (int64_t)1 << log2n;
    scl_path* cur = (scl_path*)calloc((size_t)list, sizeof(scl_path));
    scl_path* nxt = (scl_path*)calloc((size_t)list, sizeof(scl_path));
    for (int k = 0; k < list; ++k) {
        cur[k].a = (float*)calloc((size_t)n, sizeof(float));
        cur[k].u = (uint8_t*)calloc((size_t)n, 1);
        nxt[k].a = (float*)calloc((size_t)n, sizeof(float));
        nxt[k].u = (uint8_t*)calloc((size_t)n, 1);
    }
    uint8_t* beta = (uint8_t*)malloc((size_t)n);
    float* lam = (float*)malloc(sizeof(float) * (size_t)list);
    scl_cand* cand = (scl_cand*)malloc(sizeof(scl_cand) * 2 * (size_t)list);
    int active = 1;
    cur[0].pm = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < active; ++k) lam[k] = scl_leaf(&cur[k], llr, log2n, i, beta);
        if (frozen[i]) {
            const int b = fval[i];
            for (int k = 0; k < active; ++k) {
                if (b != (lam[k] < 0.0f)) cur[k].pm = cur[k].pm + fabsf(lam[k]);
                cur[k].u[i] = (uint8_t)b;
            }
            continue;
        }
        int nc = 0;
        for (int k = 0; k < active; ++k)
            for (int b = 0; b < 2; ++b) {
                scl_cand c = {cur[k].pm, k, b};
                if (b != (lam[k] < 0.0f)) c.pm = cur[k].pm + fabsf(lam[k]);
                /* insertion into the ordered list */
                int at = nc++;
                while (at > 0 && scl_before(&c, &cand[at - 1])) {
                    cand[at] = cand[at - 1];
                    --at;
                }
                cand[at] = c;
            }
        const int keep = nc < list ? nc : list;
        for (int k = 0; k < keep; ++k) {
            const scl_path* par = &cur[cand[k].parent];
            memcpy(nxt[k].a, par->a, sizeof(float) * (size_t)n);
            memcpy(nxt[k].u, par->u, (size_t)i);
            nxt[k].u[i] = (uint8_t)cand[k].bit;
            nxt[k].pm = cand[k].pm;
        }
        scl_path* t = cur;
        cur = nxt;
        nxt = t;
        active = keep;
    }
    int best = 0;
    for (int k = 1; k < active; ++k)
        if (cur[k].pm < cur[best].pm) best = k;
    memcpy(u_hat, cur[best].u, (size_t)n);
    if (pm_out) *pm_out = cur[best].pm;
    for (int k = 0; k < list; ++k) {
        free(cur[k].a);
        free(cur[k].u);
        free(nxt[k].a);
        free(nxt[k].u);
    }
    free(cur);
    free(nxt);
    free(beta);
    free(lam);
    free(cand);
    return 0;
}

float oracle_f_minsum(float a, float b) { return f_minsum(a, b); }
float oracle_g_f32(float a, float b, int u) { return g_f32(a, b, u); }
double oracle_f_boxplus(double a, double b) { return f_boxplus(a, b); }
int32_t oracle_f_fixed(int kind, int32_t a, int32_t b, const int32_t* table, int len) {
    fx_ctx c;
    memset(&c, 0, sizeof c);
    c.kind = kind;
    c.max = kind == 2 ? FIXED8_MAX : FIXED_MAX;
    c.table = table;
    c.len = len;
    return fx_f(&c, a, b);
}

/* ------------------------------------------------------------------------ */
/* Many frames, one frame per thread (the CPU baseline).                    */
/* Frame k reads llr + k*N, frozen + (shared ? 0 : k*N), fval + k*N and     */
/* writes u_hat + k*N.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int log2n, boxplus, n_frames, shared_frozen, n_threads, tid;
    const float* llr;
    const uint8_t* frozen;
    const uint8_t* fval;
    uint8_t* u_hat;
} batch_job;

static void* batch_worker(void* p) {
    batch_job* j = (batch_job*)p;
    int64_t n = (int64_t)1 << j->log2n;
    for (int k = j->tid; k < j->n_frames; k += j->n_threads) {
        const uint8_t* fz = j->frozen + (j->shared_frozen ? 0 : (int64_t)k * n);
        oracle_sc_decode(j->log2n, j->boxplus, j->llr + (int64_t)k * n, fz,
                         j->fval + (int64_t)k * n, NULL, j->u_hat + (int64_t)k * n, NULL, NULL);
    }
    return NULL;
}

int oracle_sc_decode_batch(int log2n, int boxplus, int n_frames, int shared_frozen,
                           const float* llr, const uint8_t* frozen, const uint8_t* fval,
                           uint8_t* u_hat, int n_threads) {
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    batch_job jobs[256];
    for (int t = 0; t < n_threads; ++t) {
        jobs[t].log2n = log2n;
        jobs[t].boxplus = boxplus;
        jobs[t].n_frames = n_frames;
        jobs[t].shared_frozen = shared_frozen;
        jobs[t].n_threads = n_threads;
        jobs[t].tid = t;
        jobs[t].llr = llr;
        jobs[t].frozen = frozen;
        jobs[t].fval = fval;
        jobs[t].u_hat = u_hat;
        pthread_create(&th[t], NULL, batch_worker, &jobs[t]);
    }
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    return 0;
}
