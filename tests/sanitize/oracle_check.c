/* Exercises the CPU oracle's entry points at small ring degrees, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py):
 * any invalid access, leak-free misuse or undefined operation aborts with a
 * report.  Prints the decrypted errors of a few results as a sanity check. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_ctx orc_ctx;
typedef struct orc_ct orc_ct;
orc_ctx *orc_ctx_create(int logN, int L, int K, int alpha, int h, double sigma, int log_delta, int q0_bits,
                        int p_bits);
orc_ctx *orc_ctx_create_bts(int logN, int l_after, int n_stc, int n_evm, int n_cts, int bts_bits, int K, int alpha,
                            int h, double sigma, int log_delta, int q0_bits, int p_bits);
void orc_ctx_free(orc_ctx *c);
int orc_keygen(orc_ctx *c, uint64_t seed, const int32_t *galois, int ngal);
int orc_galois_rot(orc_ctx *c, int k);
orc_ct *orc_encrypt(orc_ctx *c, const double *x, int nslots, int level, double scale, uint64_t seed);
int orc_decrypt(orc_ctx *c, const orc_ct *ct, double *re, double *im);
void orc_ct_free(orc_ct *ct);
orc_ct *orc_add(orc_ctx *c, const orc_ct *a, const orc_ct *b);
orc_ct *orc_sub(orc_ctx *c, const orc_ct *a, const orc_ct *b);
orc_ct *orc_mul_const_down(orc_ctx *c, const orc_ct *a, double value);
orc_ct *orc_hmult(orc_ctx *c, const orc_ct *a, const orc_ct *b);
orc_ct *orc_mult_rs(orc_ctx *c, const orc_ct *a, const orc_ct *b);
orc_ct *orc_rescale(orc_ctx *c, const orc_ct *a);
orc_ct *orc_rotate(orc_ctx *c, const orc_ct *a, int k);
orc_ct *orc_conjugate(orc_ctx *c, const orc_ct *a);
int orc_rotate_hoisted(orc_ctx *c, const orc_ct *a, const int *steps, int n, orc_ct **outs);
int orc_cheb_coeffs_invsqrt(int d, double a, double b, double *out);
orc_ct *orc_cheb_eval(orc_ctx *c, const orc_ct *x, const double *cf, int d, double a, double b);
orc_ct *orc_invsqrt(orc_ctx *c, const orc_ct *x, int d, int iters, double a, double b, int literal, int64_t bts_bound,
                    int pre_bts, double B);
int orc_bts_config(orc_ctx *c, double Kp, int r, int deg);
int orc_bts_rotations(orc_ctx *c, int32_t *out, int max);
orc_ct *orc_bootstrap(orc_ctx *c, const orc_ct *a, int64_t M);
void orc_shake256(const uint8_t *in, size_t len, uint8_t *out, size_t outlen);
const char *orc_last_error(void);

static double max_rel(orc_ctx *c, const orc_ct *y, const double *want, int n) {
    double *re = malloc(sizeof(double) * n), *im = malloc(sizeof(double) * n), m = 0;
    orc_decrypt(c, y, re, im);
    for (int i = 0; i < n; i++) {
        double e = fabs(re[i] - want[i]) / fabs(want[i]);
        if (e > m) m = e;
    }
    free(re); free(im);
    return m;
}

int main(void) {
    uint8_t msg[300], out[500];
    for (int i = 0; i < 300; i++) msg[i] = (uint8_t)(i * 7);
    orc_shake256(msg, 300, out, 500);

    /* plain chain, N = 2^8 */
    orc_ctx *c = orc_ctx_create(8, 9, 1, 1, 0, 3.2, 40, 60, 60);
    if (!c) return 2;
    const int n = 128;
    int32_t gal[3] = {orc_galois_rot(c, 1), orc_galois_rot(c, -3), 2 * 256 - 1};
    if (orc_keygen(c, 7, gal, 3)) return 3;
    double x[128], inv[128];
    for (int i = 0; i < n; i++) {
        x[i] = pow(2.0, -8.0 * (double)(i + 1) / n);
        inv[i] = 1.0 / sqrt(x[i]);
    }
    orc_ct *a = orc_encrypt(c, x, n, 9, ldexp(1.0, 50), 3);
    orc_ct *s = orc_add(c, a, a), *d = orc_sub(c, s, a);
    orc_ct *h = orc_mul_const_down(c, a, 0.5);
    orc_ct *p = orc_hmult(c, h, h), *r = orc_rescale(c, p), *m = orc_mult_rs(c, h, h);
    orc_ct *ro = orc_rotate(c, a, 1), *cj = orc_conjugate(c, a);
    int steps[3] = {0, 1, -3};
    orc_ct *hs[3] = {0};
    if (orc_rotate_hoisted(c, a, steps, 3, hs)) return 4;
    double cf[32];
    orc_cheb_coeffs_invsqrt(31, ldexp(1.0, -8), 1.0, cf);
    orc_ct *y = orc_cheb_eval(c, a, cf, 31, ldexp(1.0, -8), 1.0);
    orc_ct *z = orc_invsqrt(c, a, 15, 2, ldexp(1.0, -8), 1.0, 0, 0, 0, 0.0);
    orc_ct *zb = orc_invsqrt(c, a, 14, 1, ldexp(1.0, -8), 1.0, 0, 0, 0, 100.0);
    if (!s || !d || !h || !p || !r || !m || !ro || !cj || !y || !z || !zb) return 5;
    printf("plain: cheb(31) max rel err %.3g, invsqrt(15,2) max rel err %.3g\n", max_rel(c, y, inv, n),
           max_rel(c, z, inv, n));
    fflush(stdout);
    orc_ct *all[] = {a, s, d, h, p, r, m, ro, cj, y, z, zb, hs[0], hs[1], hs[2]};
    for (unsigned i = 0; i < sizeof(all) / sizeof(all[0]); i++) orc_ct_free(all[i]);
    orc_ctx_free(c);

    /* bootstrapping chain, N = 2^8 */
    orc_ctx *b = orc_ctx_create_bts(8, 5, 3, 9, 3, 52, 2, 2, 16, 3.2, 40, 60, 60);
    if (!b || orc_bts_config(b, 25.0, 4, 31)) return 6;
    int32_t rots[256];
    int nr = orc_bts_rotations(b, rots, 256);
    if (nr < 0) return 7;
    int32_t *bg = malloc(sizeof(int32_t) * (nr + 1));
    for (int i = 0; i < nr; i++) bg[i] = orc_galois_rot(b, rots[i]);
    bg[nr] = 2 * 256 - 1;
    if (orc_keygen(b, 9, bg, nr + 1)) return 8;
    free(bg);
    orc_ct *bx = orc_encrypt(b, x, n, 5, ldexp(1.0, 50), 5);
    orc_ct *bl = orc_invsqrt(b, bx, 15, 3, ldexp(1.0, -8), 1.0, 1, 0, 0, 0.0);
    orc_ct *bp = orc_invsqrt(b, bx, 7, 2, ldexp(1.0, -8), 1.0, 0, 0, 1, 0.0);
    orc_ct *bb = orc_bootstrap(b, bx, 16);
    if (!bx || !bl || !bp || !bb) {
        printf("bootstrapping step failed: %d %d %d %d: %s\n", !bx, !bl, !bp, !bb, orc_last_error());
        return 9;
    }
    printf("bootstrapping: literal (15,3) max rel err %.3g, bootstrap of x max rel err %.3g\n",
           max_rel(b, bl, inv, n), max_rel(b, bb, x, n));
    orc_ct_free(bx); orc_ct_free(bl); orc_ct_free(bp); orc_ct_free(bb);
    orc_ctx_free(b);
    return 0;
}
