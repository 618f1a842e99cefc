/*
 * ckks_oracle.c -- plain, slow, single-threaded CPU oracle for the encrypted
 * inverse square root (paper: Alg. 1 "CryptoInvSqrt", Newton step of §2.2,
 * Chebyshev initial value of §2.3) and for the RNS-CKKS arithmetic it runs on
 * (the operations Add/Sub/Mul_P/Mul_C/BTS named in §2.1; the scheme itself
 * is the CKKS scheme the paper cites, in its RNS form with hybrid key
 * switching).
 *
 * THIS IS TEST INFRASTRUCTURE.  It exists only to check the GPU library.
 * Only the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant
 * generator with the GPU library: every routine here is written from the
 * mathematical definition, with no blocking, fusion or reordering beyond what
 * that definition states.
 *
 * Precision rules:
 *   - modular arithmetic: exact, a*b mod q through unsigned __int128 '%';
 *   - encode / decode / Chebyshev coefficients / linear-transform diagonals:
 *     __float128 (113-bit mantissa) and rounded only at the end, so that
 *     every integer decided by floating point is the correctly rounded value
 *     of the exact real number except with negligible probability;
 *   - scale bookkeeping: plain IEEE binary64, each formula evaluated in the
 *     order written in the comment next to it (build with -ffp-contract=off).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <quadmath.h>

typedef unsigned __int128 u128;
typedef __int128 i128;
typedef __float128 f128;

/* ------------------------------------------------------------------------ */
/* Error reporting                                                           */
/* ------------------------------------------------------------------------ */
static char g_err[256];
static void set_err(const char *m) { strncpy(g_err, m, sizeof(g_err) - 1); }
const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* Modular arithmetic (exact)                                                */
/* ------------------------------------------------------------------------ */
static inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * b) % q);
}
static inline uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    uint64_t s = a + b;            /* q < 2^62, no overflow */
    return s >= q ? s - q : s;
}
static inline uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
    return a >= b ? a - b : a + q - b;
}
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }
/* signed integer -> residue in [0, q) */
static inline uint64_t smod(int64_t v, uint64_t q) {
    if (v >= 0) return (uint64_t)v % q;
    uint64_t m = (uint64_t)(-(v + 1)) % q;      /* -(v+1) >= 0, avoids INT64_MIN */
    return (q - 1 - m);
}

/* ------------------------------------------------------------------------ */
/* Primality: Miller-Rabin with the fixed base set {2..37}, which is a       */
/* deterministic test for every n < 3.3e24 (so for every 64-bit n).          */
/* ------------------------------------------------------------------------ */
int orc_is_prime(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* SHAKE-256 (FIPS 202), written from the Keccak-f[1600] definition.         */
/* ------------------------------------------------------------------------ */
static uint64_t keccak_rc[24];
static int keccak_rot[25];
static int keccak_ready = 0;

/* rc(t) of FIPS 202 §3.2.5: the output bit of an 8-bit LFSR */
static int keccak_rc_bit(int t) {
    if (t % 255 == 0) return 1;
    unsigned R = 1; /* bit i of R is R[i]; R = 10000000 means R[0] = 1 */
    for (int i = 1; i <= t % 255; i++) {
        unsigned r8;
        R <<= 1;              /* R = 0 || R, R[8] is the old R[7] */
        r8 = (R >> 8) & 1;
        R ^= r8;              /* R[0] ^= R[8] */
        R ^= r8 << 4;
        R ^= r8 << 5;
        R ^= r8 << 6;
        R &= 0xFF;
    }
    return R & 1;
}
static void keccak_init_tables(void) {
    if (keccak_ready) return;
    for (int ir = 0; ir < 24; ir++) {
        uint64_t rc = 0;
        for (int j = 0; j <= 6; j++)
            if (keccak_rc_bit(j + 7 * ir)) rc |= (uint64_t)1 << ((1 << j) - 1);
        keccak_rc[ir] = rc;
    }
    /* rho offsets, FIPS 202 §3.2.2 */
    for (int i = 0; i < 25; i++) keccak_rot[i] = 0;
    int x = 1, y = 0;
    for (int t = 0; t < 24; t++) {
        keccak_rot[x + 5 * y] = ((t + 1) * (t + 2) / 2) % 64;
        int nx = y, ny = (2 * x + 3 * y) % 5;
        x = nx; y = ny;
    }
    keccak_ready = 1;
}
static inline uint64_t rotl64(uint64_t v, int r) { return r ? (v << r) | (v >> (64 - r)) : v; }
static void keccak_f1600(uint64_t A[25]) {
    for (int ir = 0; ir < 24; ir++) {
        uint64_t C[5], D[5], B[25];
        for (int x = 0; x < 5; x++) C[x] = A[x] ^ A[x + 5] ^ A[x + 10] ^ A[x + 15] ^ A[x + 20];
        for (int x = 0; x < 5; x++) D[x] = C[(x + 4) % 5] ^ rotl64(C[(x + 1) % 5], 1);
        for (int i = 0; i < 25; i++) A[i] ^= D[i % 5];
        /* rho + pi: B[y, 2x+3y] = rot(A[x,y]) */
        for (int x = 0; x < 5; x++)
            for (int y = 0; y < 5; y++)
                B[y + 5 * ((2 * x + 3 * y) % 5)] = rotl64(A[x + 5 * y], keccak_rot[x + 5 * y]);
        for (int x = 0; x < 5; x++)
            for (int y = 0; y < 5; y++)
                A[x + 5 * y] = B[x + 5 * y] ^ ((~B[(x + 1) % 5 + 5 * y]) & B[(x + 2) % 5 + 5 * y]);
        A[0] ^= keccak_rc[ir];
    }
}
typedef struct { uint64_t st[25]; uint8_t buf[136]; int pos; } xof_t;
#define SHAKE_RATE 136
static void xof_absorb_final(xof_t *x, const uint8_t *in, size_t len) {
    keccak_init_tables();
    memset(x, 0, sizeof(*x));
    uint8_t block[SHAKE_RATE];
    while (len >= SHAKE_RATE) {
        for (int i = 0; i < SHAKE_RATE / 8; i++) {
            uint64_t w = 0;
            for (int b = 0; b < 8; b++) w |= (uint64_t)in[8 * i + b] << (8 * b);
            x->st[i] ^= w;
        }
        keccak_f1600(x->st);
        in += SHAKE_RATE; len -= SHAKE_RATE;
    }
    memset(block, 0, sizeof(block));
    memcpy(block, in, len);
    block[len] ^= 0x1F;                 /* SHAKE domain bits + first pad bit */
    block[SHAKE_RATE - 1] ^= 0x80;      /* last pad bit */
    for (int i = 0; i < SHAKE_RATE / 8; i++) {
        uint64_t w = 0;
        for (int b = 0; b < 8; b++) w |= (uint64_t)block[8 * i + b] << (8 * b);
        x->st[i] ^= w;
    }
    x->pos = SHAKE_RATE; /* force a permutation before the first squeeze */
}
static uint8_t xof_byte(xof_t *x) {
    if (x->pos == SHAKE_RATE) {
        keccak_f1600(x->st);
        for (int i = 0; i < SHAKE_RATE / 8; i++)
            for (int b = 0; b < 8; b++) x->buf[8 * i + b] = (uint8_t)(x->st[i] >> (8 * b));
        x->pos = 0;
    }
    return x->buf[x->pos++];
}
/*
 * Note on the squeeze: after absorbing the final padded block the sponge
 * applies f once (inside xof_byte, the first time) and outputs the first
 * rate bytes; every further block applies f again.
 */
static void xof_init(xof_t *x, uint64_t seed, uint64_t tag) {
    uint8_t in[16];
    for (int b = 0; b < 8; b++) in[b] = (uint8_t)(seed >> (8 * b));
    for (int b = 0; b < 8; b++) in[8 + b] = (uint8_t)(tag >> (8 * b));
    xof_absorb_final(x, in, 16);
}
static uint64_t xof_u64(xof_t *x) {
    uint64_t w = 0;
    for (int b = 0; b < 8; b++) w |= (uint64_t)xof_byte(x) << (8 * b);
    return w;
}
static uint32_t xof_u32(xof_t *x) {
    uint32_t w = 0;
    for (int b = 0; b < 4; b++) w |= (uint32_t)xof_byte(x) << (8 * b);
    return w;
}
/* exposed for the byte-equality pin against hashlib.shake_256 */
void orc_shake256(const uint8_t *in, size_t len, uint8_t *out, size_t outlen) {
    xof_t x;
    keccak_init_tables();
    /* absorb whole blocks then the padded tail */
    xof_absorb_final(&x, in, len);
    for (size_t i = 0; i < outlen; i++) out[i] = xof_byte(&x);
}

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int galois;              /* 0 = relinearisation key */
    uint64_t *k;             /* [dnum][2][nprimes][N] */
} evk_t;

typedef struct orc_ctx {
    int logN, N, n;          /* ring degree, slots */
    int L, K, alpha, dnum, h;
    double sigma;
    int log_delta;
    int np;                  /* L+1+K */
    uint64_t *q;             /* [np]  q_0..q_L, p_0..p_{K-1} */
    uint64_t *psi_br;        /* [np][N] psi^br(k) */
    uint64_t *ipsi_br;       /* [np][N] psi^-br(k) */
    uint64_t *ninv;          /* [np] */
    double *ladder;          /* [L+1] canonical scale per level */
    /* bootstrapping-shaped chain (all zero for a plain chain) */
    int l_after, n_stc, n_evm, n_cts, bts_bits;
    struct bts_plan *bts;    /* set by orc_bts_config */
    uint64_t cdt[64];        /* Gaussian CDT thresholds (53-bit) */
    int cdt_len;
    /* keys */
    int have_sk;
    int8_t *s;               /* [N] */
    uint64_t *s_ntt;         /* [np][N] */
    uint64_t *pk;            /* [2][L+1][N] */
    evk_t relin;
    evk_t *rot;              /* rotation / conjugation keys */
    int nrot;
} orc_ctx;

typedef struct orc_ct {
    int level;
    double scale;
    uint64_t *c;             /* [2][level+1][N], NTT domain */
} orc_ct;

static int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* smallest g >= 2 such that psi = g^((q-1)/2N) has psi^N = -1 (order 2N) */
static uint64_t find_psi(uint64_t q, int N) {
    for (uint64_t g = 2;; g++) {
        uint64_t psi = powmod(g, (q - 1) / (2 * (uint64_t)N), q);
        if (powmod(psi, (uint64_t)N, q) == q - 1) return psi;
    }
}
uint64_t orc_psi(uint64_t q, int N) { return find_psi(q, N); }

static int prime_used(const uint64_t *list, int cnt, uint64_t c) {
    for (int i = 0; i < cnt; i++) if (list[i] == c) return 1;
    return 0;
}

/*
 * Prime chain (a reading: the paper gives only totals).
 *   q_0 : largest prime below 2^q0_bits with q = 1 mod 2N.
 *   Computation levels A..1 (A = L for a plain chain, A = l_after for a
 *   bootstrapping chain): chosen top-down.  The canonical scale of level A
 *   is S_A = 2^log_delta and S_{l-1} = (S_l * S_l) / q_l.  q_l is the unused
 *   prime = 1 mod 2N closest to T = (S_l*S_l)/2^log_delta (first prime below
 *   T and first prime above T; the closer one wins, ties go to the lower).
 *   This keeps every S_l close to 2^log_delta, so a product of two level-l
 *   ciphertexts that carry S_l lands exactly on S_{l-1} after the rescale.
 * A bootstrapping chain adds, above level A, the levels that bootstrapping
 * consumes (the ModRaised ciphertext enters at level L and leaves at A):
 *   levels A+1..A+n_stc        SlotToCoeff: q_l = unused prime closest to
 *                              2^log_delta (l ascending), S_l = 2^log_delta;
 *   levels A+n_stc+1..E        EvalMod, E = A+n_stc+n_evm: the same adaptive
 *                              rule as the computation levels, run top-down
 *                              from S_E = 2^bts_bits (this also sets S at
 *                              level A+n_stc, the EvalMod output);
 *   levels E+1..L              CoeffToSlot: unused prime closest to
 *                              2^bts_bits (l ascending), S_l = 2^bts_bits.
 *   Selection order: q_0, computation levels, EvalMod, SlotToCoeff,
 *   CoeffToSlot, then the special primes.
 *   p_0..p_{K-1}: the next unused primes = 1 mod 2N below 2^p_bits (descending).
 */
static uint64_t closest_prime(uint64_t M, double T, const uint64_t *chosen, int nch) {
    uint64_t Ti = (uint64_t)floor(T);
    uint64_t lo = Ti - ((Ti - 1) % M);          /* first candidate = 1 mod M at or below Ti */
    uint64_t hi = lo + M;
    while (!(orc_is_prime(lo) && !prime_used(chosen, nch, lo))) lo -= M;
    while (!(orc_is_prime(hi) && !prime_used(chosen, nch, hi))) hi += M;
    double dlo = T - (double)lo, dhi = (double)hi - T;
    return (dhi < dlo) ? hi : lo;
}
/* adaptive top-down run over levels top..bot+1 starting from S_top = D */
static void adaptive_run(orc_ctx *c, int top, int bot, double D, uint64_t *chosen, int *nch) {
    uint64_t M = 2 * (uint64_t)c->N;
    double S = D;
    c->ladder[top] = S;
    for (int l = top; l > bot; l--) {
        double T = (S * S) / D;
        uint64_t pick = closest_prime(M, T, chosen, *nch);
        c->q[l] = pick;
        chosen[(*nch)++] = pick;
        S = (S * S) / (double)pick;
        c->ladder[l - 1] = S;
    }
}
static int gen_primes(orc_ctx *c, int q0_bits, int p_bits) {
    uint64_t M = 2 * (uint64_t)c->N;
    uint64_t *q = c->q;
    uint64_t top = ((uint64_t)1 << q0_bits);
    uint64_t cand = top - ((top - 1) % M);      /* largest x <= top with x = 1 mod M */
    if (cand >= top) cand -= M;
    while (!orc_is_prime(cand)) cand -= M;
    q[0] = cand;
    uint64_t chosen[256];
    chosen[0] = q[0];
    int nch = 1;
    const double Dc = ldexp(1.0, c->log_delta);
    const int A = c->l_after;
    adaptive_run(c, A, 0, Dc, chosen, &nch);
    if (c->n_evm > 0) {
        const double Db = ldexp(1.0, c->bts_bits);
        const int E = A + c->n_stc + c->n_evm;
        adaptive_run(c, E, A + c->n_stc, Db, chosen, &nch);
        for (int l = A + 1; l <= A + c->n_stc; l++) {
            q[l] = closest_prime(M, Dc, chosen, nch);
            chosen[nch++] = q[l];
            if (l < A + c->n_stc) c->ladder[l] = Dc;
        }
        for (int l = E + 1; l <= c->L; l++) {
            q[l] = closest_prime(M, Db, chosen, nch);
            chosen[nch++] = q[l];
            c->ladder[l] = Db;
        }
    }
    int cnt = c->L + 1;
    uint64_t ptop = ((uint64_t)1 << p_bits);
    uint64_t pc = ptop - ((ptop - 1) % M);
    if (pc >= ptop) pc -= M;
    for (int k = 0; k < c->K; k++) {
        while (!(orc_is_prime(pc) && !prime_used(chosen, nch, pc))) pc -= M;
        q[cnt++] = pc;
        chosen[nch++] = pc;
        pc -= M;
    }
    return 0;
}

/*
 * Discrete Gaussian CDT (sigma, tail cut at 6.25 sigma rounded up):
 *   rho(j) = exp(-(j*j) / (2*sigma*sigma)),   j = 0..J
 *   Z      = rho(0) + 2*(rho(1) + ... + rho(J))      (summed for j ascending)
 *   F(k)   = (rho(0) + 2*(rho(1)+...+rho(k))) / Z
 *   T[k]   = (uint64)(F(k) * 2^53) for k < J, T[J] = 2^53.
 * A sample draws w (64 bits), u = w >> 11, |e| = min{k : u < T[k]},
 * sign = w & 1 (1 -> negative).
 */
static void build_cdt(orc_ctx *c) {
    int J = (int)ceil(6.25 * c->sigma);
    if (J > 63) J = 63;
    double den = 2.0 * c->sigma * c->sigma;
    double rho[64];
    for (int j = 0; j <= J; j++) rho[j] = exp(-((double)j * (double)j) / den);
    double tail = 0.0;
    for (int j = 1; j <= J; j++) tail += rho[j];
    double Z = rho[0] + 2.0 * tail;
    double part = 0.0;
    for (int k = 0; k < J; k++) {
        if (k >= 1) part += rho[k];
        double F = (rho[0] + 2.0 * part) / Z;
        c->cdt[k] = (uint64_t)(F * 9007199254740992.0);
    }
    c->cdt[J] = (uint64_t)1 << 53;
    c->cdt_len = J + 1;
}
int orc_cdt(orc_ctx *c, uint64_t *out) {
    for (int i = 0; i < c->cdt_len; i++) out[i] = c->cdt[i];
    return c->cdt_len;
}

orc_ctx *orc_ctx_create_bts(int logN, int l_after, int n_stc, int n_evm, int n_cts, int bts_bits,
                            int K, int alpha, int h, double sigma, int log_delta, int q0_bits, int p_bits) {
    const int bts = n_evm > 0;
    const int L = l_after + n_stc + n_evm + n_cts;
    if (logN < 2 || logN > 17 || l_after < 1 || L > 60 || K < 1 || alpha < 1 ||
        q0_bits > 61 || p_bits > 61 || log_delta < 20 || log_delta > 58 ||
        (bts && (n_stc < 1 || n_cts < 1 || bts_bits < 20 || bts_bits > 61 || logN < 4)) ||
        (!bts && (n_stc || n_cts))) {
        set_err("bad parameters");
        return NULL;
    }
    orc_ctx *c = calloc(1, sizeof(orc_ctx));
    c->logN = logN; c->N = 1 << logN; c->n = c->N / 2;
    c->L = L; c->K = K; c->alpha = alpha; c->h = h; c->sigma = sigma;
    c->log_delta = log_delta;
    c->l_after = l_after; c->n_stc = n_stc; c->n_evm = n_evm; c->n_cts = n_cts; c->bts_bits = bts_bits;
    c->dnum = (L + 1 + alpha - 1) / alpha;
    c->np = L + 1 + K;
    c->q = calloc(c->np, sizeof(uint64_t));
    c->ladder = calloc(L + 1, sizeof(double));
    gen_primes(c, q0_bits, p_bits);
    size_t N = c->N;
    c->psi_br = malloc(sizeof(uint64_t) * c->np * N);
    c->ipsi_br = malloc(sizeof(uint64_t) * c->np * N);
    c->ninv = malloc(sizeof(uint64_t) * c->np);
    for (int i = 0; i < c->np; i++) {
        uint64_t q = c->q[i];
        uint64_t psi = find_psi(q, c->N);
        uint64_t ipsi = invmod(psi, q);
        for (int k = 0; k < c->N; k++) {
            int e = bitrev(k, logN);
            c->psi_br[i * N + k] = powmod(psi, (uint64_t)e, q);
            c->ipsi_br[i * N + k] = powmod(ipsi, (uint64_t)e, q);
        }
        c->ninv[i] = invmod((uint64_t)c->N, q);
    }
    build_cdt(c);
    return c;
}
orc_ctx *orc_ctx_create(int logN, int L, int K, int alpha, int h, double sigma,
                        int log_delta, int q0_bits, int p_bits) {
    return orc_ctx_create_bts(logN, L, 0, 0, 0, 0, K, alpha, h, sigma, log_delta, q0_bits, p_bits);
}

static void evk_free(evk_t *e) { free(e->k); e->k = NULL; }
struct bts_plan;
static void bts_plan_free(struct bts_plan *b);
void orc_ctx_free(orc_ctx *c) {
    if (!c) return;
    free(c->q); free(c->psi_br); free(c->ipsi_br); free(c->ninv); free(c->ladder);
    free(c->s); free(c->s_ntt); free(c->pk);
    evk_free(&c->relin);
    for (int i = 0; i < c->nrot; i++) evk_free(&c->rot[i]);
    free(c->rot);
    bts_plan_free(c->bts);
    free(c);
}
int orc_ctx_info(orc_ctx *c, uint64_t *primes, double *ladder) {
    if (primes) memcpy(primes, c->q, sizeof(uint64_t) * c->np);
    if (ladder) memcpy(ladder, c->ladder, sizeof(double) * (c->L + 1));
    return c->np;
}
int orc_dnum(orc_ctx *c) { return c->dnum; }

/* ------------------------------------------------------------------------ */
/* NTT.  Definition: NTT(a)[j] = sum_i a_i * psi^((2*br(j)+1)*i) mod q,      */
/* i.e. evaluation of a(X) at the odd powers of psi, stored in bit-reversed  */
/* order.  Computed with the textbook Cooley-Tukey (forward) and             */
/* Gentleman-Sande (inverse) iterations, merged negacyclic twist.            */
/* ------------------------------------------------------------------------ */
static void ntt_fwd(const orc_ctx *c, int pi, uint64_t *a) {
    int N = c->N;
    uint64_t q = c->q[pi];
    const uint64_t *W = c->psi_br + (size_t)pi * N;
    int t = N;
    for (int m = 1; m < N; m <<= 1) {
        t >>= 1;
        for (int i = 0; i < m; i++) {
            int j1 = 2 * i * t;
            uint64_t S = W[m + i];
            for (int j = j1; j < j1 + t; j++) {
                uint64_t U = a[j], V = mulmod(a[j + t], S, q);
                a[j] = addmod(U, V, q);
                a[j + t] = submod(U, V, q);
            }
        }
    }
}
static void ntt_inv(const orc_ctx *c, int pi, uint64_t *a) {
    int N = c->N;
    uint64_t q = c->q[pi];
    const uint64_t *W = c->ipsi_br + (size_t)pi * N;
    int t = 1;
    for (int m = N; m > 1; m >>= 1) {
        int h = m >> 1, j1 = 0;
        for (int i = 0; i < h; i++) {
            uint64_t S = W[h + i];
            for (int j = j1; j < j1 + t; j++) {
                uint64_t U = a[j], V = a[j + t];
                a[j] = addmod(U, V, q);
                a[j + t] = mulmod(submod(U, V, q), S, q);
            }
            j1 += 2 * t;
        }
        t <<= 1;
    }
    for (int j = 0; j < N; j++) a[j] = mulmod(a[j], c->ninv[pi], q);
}
/* exported for tests: prime index pi in the extended basis */
void orc_ntt(orc_ctx *c, int pi, uint64_t *a) { ntt_fwd(c, pi, a); }
void orc_intt(orc_ctx *c, int pi, uint64_t *a) { ntt_inv(c, pi, a); }

/* ------------------------------------------------------------------------ */
/* Sampling                                                                  */
/* ------------------------------------------------------------------------ */
enum { TAG_SK = 1, TAG_PK_A = 2, TAG_PK_E = 3, TAG_EVK_A = 4, TAG_EVK_E = 5,
       TAG_ENC_V = 6, TAG_ENC_E0 = 7, TAG_ENC_E1 = 8 };
static uint64_t mk_tag(int kind, int galois, int digit) {
    return ((uint64_t)kind << 56) | ((uint64_t)(uint32_t)galois << 16) | (uint64_t)(uint16_t)digit;
}
/* uniform residues for the primes idx[0..cnt): per prime, N values by
 * rejection of 64-bit words masked to bitlen(q) */
static void sample_uniform(const orc_ctx *c, xof_t *x, const int *idx, int cnt, uint64_t *out) {
    for (int t = 0; t < cnt; t++) {
        uint64_t q = c->q[idx[t]];
        int bl = 64 - __builtin_clzll(q);
        uint64_t mask = (bl == 64) ? ~(uint64_t)0 : (((uint64_t)1 << bl) - 1);
        for (int j = 0; j < c->N; j++) {
            uint64_t w;
            do { w = xof_u64(x) & mask; } while (w >= q);
            out[(size_t)t * c->N + j] = w;
        }
    }
}
static void sample_ternary(const orc_ctx *c, xof_t *x, int8_t *out) {
    for (int j = 0; j < c->N; j++) {
        uint8_t b;
        do { b = xof_byte(x); } while (b == 255);
        out[j] = (int8_t)((int)(b % 3) - 1);
    }
}
static void sample_hwt(const orc_ctx *c, xof_t *x, int h, int8_t *out) {
    memset(out, 0, c->N);
    int cnt = 0;
    while (cnt < h) {
        uint32_t r = xof_u32(x) & (uint32_t)(c->N - 1);
        if (out[r] != 0) continue;
        uint8_t b = xof_byte(x);
        out[r] = (b & 1) ? -1 : 1;
        cnt++;
    }
}
static void sample_gauss(const orc_ctx *c, xof_t *x, int64_t *out) {
    for (int j = 0; j < c->N; j++) {
        uint64_t w = xof_u64(x);
        uint64_t u = w >> 11;
        int k = 0;
        while (k < c->cdt_len - 1 && !(u < c->cdt[k])) k++;
        int64_t e = k;
        if (k != 0 && (w & 1)) e = -e;
        out[j] = e;
    }
}
/* small signed polynomial -> NTT residues for primes idx[] */
static void small_to_ntt_i64(const orc_ctx *c, const int64_t *v, const int *idx, int cnt, uint64_t *out) {
    for (int t = 0; t < cnt; t++) {
        uint64_t q = c->q[idx[t]];
        uint64_t *o = out + (size_t)t * c->N;
        for (int j = 0; j < c->N; j++) o[j] = smod(v[j], q);
        ntt_fwd(c, idx[t], o);
    }
}
static void small_to_ntt_i8(const orc_ctx *c, const int8_t *v, const int *idx, int cnt, uint64_t *out) {
    for (int t = 0; t < cnt; t++) {
        uint64_t q = c->q[idx[t]];
        uint64_t *o = out + (size_t)t * c->N;
        for (int j = 0; j < c->N; j++) o[j] = smod(v[j], q);
        ntt_fwd(c, idx[t], o);
    }
}

/* ------------------------------------------------------------------------ */
/* Automorphism X -> X^g in the NTT domain:                                  */
/*   out[j] = in[br((g*(2*br(j)+1) mod 2N - 1)/2)]                           */
/* ------------------------------------------------------------------------ */
static void automorph_idx(const orc_ctx *c, int g, int *perm) {
    int N = c->N, M = 2 * N;
    for (int j = 0; j < N; j++) {
        int e = 2 * bitrev(j, c->logN) + 1;
        int ge = (int)(((int64_t)g * e) % M);
        perm[j] = bitrev((ge - 1) / 2, c->logN);
    }
}
int orc_automorph_perm(orc_ctx *c, int g, int32_t *perm) {
    automorph_idx(c, g, (int *)perm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Key generation                                                            */
/* ------------------------------------------------------------------------ */
/*
 * Switching key from s' (NTT form over all np primes) to s, hybrid form with
 * dnum digits of alpha primes (digit j = primes jα .. min((j+1)α, L+1)-1):
 *   b_j = -a_j*s + e_j + [prime in digit j] * (P mod q) * s'  (Q primes)
 *   b_j = -a_j*s + e_j                                         (P primes)
 * stored [j][0]=b_j, [j][1]=a_j.
 */
static void make_evk(orc_ctx *c, uint64_t seed, int galois, const uint64_t *sp, evk_t *out) {
    size_t N = c->N, np = c->np;
    out->galois = galois;
    out->k = malloc(sizeof(uint64_t) * c->dnum * 2 * np * N);
    int *all = malloc(sizeof(int) * np);
    for (size_t i = 0; i < np; i++) all[i] = (int)i;
    int64_t *e = malloc(sizeof(int64_t) * N);
    uint64_t *eN = malloc(sizeof(uint64_t) * np * N);
    /* P mod q_i */
    uint64_t *Pmod = malloc(sizeof(uint64_t) * (c->L + 1));
    for (int i = 0; i <= c->L; i++) {
        uint64_t r = 1;
        for (int k = 0; k < c->K; k++) r = mulmod(r, c->q[c->L + 1 + k] % c->q[i], c->q[i]);
        Pmod[i] = r;
    }
    for (int j = 0; j < c->dnum; j++) {
        uint64_t *b = out->k + ((size_t)j * 2 + 0) * np * N;
        uint64_t *a = out->k + ((size_t)j * 2 + 1) * np * N;
        xof_t xa, xe;
        xof_init(&xa, seed, mk_tag(TAG_EVK_A, galois, j));
        sample_uniform(c, &xa, all, (int)np, a);
        xof_init(&xe, seed, mk_tag(TAG_EVK_E, galois, j));
        sample_gauss(c, &xe, e);
        small_to_ntt_i64(c, e, all, (int)np, eN);
        int lo = j * c->alpha, hi = (j + 1) * c->alpha;
        if (hi > c->L + 1) hi = c->L + 1;
        for (size_t i = 0; i < np; i++) {
            uint64_t q = c->q[i];
            for (size_t t = 0; t < N; t++) {
                uint64_t as = mulmod(a[i * N + t], c->s_ntt[i * N + t], q);
                uint64_t v = submod(eN[i * N + t], as, q);
                if ((int)i >= lo && (int)i < hi)
                    v = addmod(v, mulmod(Pmod[i], sp[i * N + t], q), q);
                b[i * N + t] = v;
            }
        }
    }
    free(all); free(e); free(eN); free(Pmod);
}

int orc_keygen(orc_ctx *c, uint64_t seed, const int32_t *galois, int ngal) {
    size_t N = c->N, np = c->np;
    int *all = malloc(sizeof(int) * np);
    for (size_t i = 0; i < np; i++) all[i] = (int)i;
    free(c->s); free(c->s_ntt); free(c->pk);
    c->s = malloc(N);
    xof_t x;
    xof_init(&x, seed, mk_tag(TAG_SK, 0, 0));
    if (c->h > 0) sample_hwt(c, &x, c->h, c->s);
    else sample_ternary(c, &x, c->s);
    c->s_ntt = malloc(sizeof(uint64_t) * np * N);
    small_to_ntt_i8(c, c->s, all, (int)np, c->s_ntt);
    /* public key over Q_L */
    int nq = c->L + 1;
    c->pk = malloc(sizeof(uint64_t) * 2 * nq * N);
    uint64_t *pk0 = c->pk, *pk1 = c->pk + nq * N;
    xof_init(&x, seed, mk_tag(TAG_PK_A, 0, 0));
    sample_uniform(c, &x, all, nq, pk1);
    int64_t *e = malloc(sizeof(int64_t) * N);
    uint64_t *eN = malloc(sizeof(uint64_t) * nq * N);
    xof_init(&x, seed, mk_tag(TAG_PK_E, 0, 0));
    sample_gauss(c, &x, e);
    small_to_ntt_i64(c, e, all, nq, eN);
    for (int i = 0; i < nq; i++)
        for (size_t t = 0; t < N; t++)
            pk0[i * N + t] = submod(eN[i * N + t], mulmod(pk1[i * N + t], c->s_ntt[i * N + t], c->q[i]), c->q[i]);
    free(e); free(eN);
    /* relinearisation key: s' = s^2 */
    uint64_t *sp = malloc(sizeof(uint64_t) * np * N);
    for (size_t i = 0; i < np; i++)
        for (size_t t = 0; t < N; t++)
            sp[i * N + t] = mulmod(c->s_ntt[i * N + t], c->s_ntt[i * N + t], c->q[i]);
    evk_free(&c->relin);
    make_evk(c, seed, 0, sp, &c->relin);
    /* galois keys: s' = s(X^g) */
    for (int i = 0; i < c->nrot; i++) evk_free(&c->rot[i]);
    free(c->rot);
    c->nrot = ngal;
    c->rot = calloc(ngal > 0 ? ngal : 1, sizeof(evk_t));
    int *perm = malloc(sizeof(int) * N);
    for (int r = 0; r < ngal; r++) {
        automorph_idx(c, galois[r], perm);
        for (size_t i = 0; i < np; i++)
            for (size_t t = 0; t < N; t++)
                sp[i * N + t] = c->s_ntt[i * N + perm[t]];
        make_evk(c, seed, galois[r], sp, &c->rot[r]);
    }
    free(perm); free(sp); free(all);
    c->have_sk = 1;
    return 0;
}
int orc_secret(orc_ctx *c, int8_t *out) {
    if (!c->have_sk) return -1;
    memcpy(out, c->s, c->N);
    return 0;
}
/* export a switching key (tests): which = -1 relin, else rotation key index */
int orc_evk_export(orc_ctx *c, int which, uint64_t *out) {
    evk_t *e = which < 0 ? &c->relin : &c->rot[which];
    memcpy(out, e->k, sizeof(uint64_t) * c->dnum * 2 * c->np * c->N);
    return 0;
}
int orc_pk_export(orc_ctx *c, uint64_t *out) {
    memcpy(out, c->pk, sizeof(uint64_t) * 2 * (c->L + 1) * c->N);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Canonical embedding in quad precision.                                    */
/*   slot j <-> root zeta^(5^j mod 2N), zeta = exp(i*pi/N), j < n = N/2.     */
/*   decode: w_k = m_k + i*m_{k+n};  z_j = sum_k w_k zeta_j^k                */
/*           (uses zeta_j^n = i since 5^j = 1 mod 4), evaluated as           */
/*           F = DFT_n^+(w_k zeta^k), z_j = F[(5^j mod 2N - 1)/4].           */
/*   encode: the exact inverse, then m = rint(scale * (Re w, Im w)).         */
/* ------------------------------------------------------------------------ */
typedef struct { f128 re, im; } cq;
static inline cq cq_mul(cq a, cq b) { cq r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cq cq_add(cq a, cq b) { cq r = {a.re + b.re, a.im + b.im}; return r; }
static inline cq cq_sub(cq a, cq b) { cq r = {a.re - b.re, a.im - b.im}; return r; }

/* root of unity exp(2*pi*i*k/M) */
static cq cq_root(int64_t k, int64_t M) {
    k %= M; if (k < 0) k += M;
    f128 ang = 2 * M_PIq * (f128)k / (f128)M;
    cq r = {cosq(ang), sinq(ang)};
    return r;
}

/* radix-2 DFT with sign s (+1: sum x_k w^{jk}, -1: conjugate roots), unnormalised */
static void dft_q(cq *x, int n, int sign) {
    int bits = 0; while ((1 << bits) < n) bits++;
    for (int i = 0; i < n; i++) {
        int r = bitrev(i, bits);
        if (r > i) { cq t = x[i]; x[i] = x[r]; x[r] = t; }
    }
    cq *W = malloc(sizeof(cq) * (n / 2 > 0 ? n / 2 : 1));
    for (int k = 0; k < n / 2; k++) { W[k] = cq_root(k, n); if (sign < 0) W[k].im = -W[k].im; }
    for (int len = 2; len <= n; len <<= 1) {
        int step = n / len;
        for (int i = 0; i < n; i += len)
            for (int j = 0; j < len / 2; j++) {
                cq u = x[i + j], v = cq_mul(x[i + j + len / 2], W[j * step]);
                x[i + j] = cq_add(u, v);
                x[i + j + len / 2] = cq_sub(u, v);
            }
    }
    free(W);
}
/* plain O(n^2) version, for the tests that pin dft_q */
void orc_dft_direct_test(int n, const double *re, const double *im, double *ore, double *oim, int sign) {
    for (int j = 0; j < n; j++) {
        cq acc = {0, 0};
        for (int k = 0; k < n; k++) {
            cq w = cq_root((int64_t)j * k * sign, n);
            cq v = {re[k], im[k]};
            acc = cq_add(acc, cq_mul(v, w));
        }
        ore[j] = (double)acc.re; oim[j] = (double)acc.im;
    }
}
void orc_dft_fast_test(int n, const double *re, const double *im, double *ore, double *oim, int sign) {
    cq *x = malloc(sizeof(cq) * n);
    for (int k = 0; k < n; k++) { x[k].re = re[k]; x[k].im = im[k]; }
    dft_q(x, n, sign);
    for (int j = 0; j < n; j++) { ore[j] = (double)x[j].re; oim[j] = (double)x[j].im; }
    free(x);
}

/* encode complex slots given in quad: out integer coefficients (int128) */
static int encode_q(const orc_ctx *c, const cq *z, f128 scale, i128 *out) {
    int n = c->n, N = c->N;
    cq *F = malloc(sizeof(cq) * n);
    uint64_t M = 2 * (uint64_t)N, e = 1;
    for (int j = 0; j < n; j++) {
        F[(e - 1) / 4] = z[j];
        e = (e * 5) % M;
    }
    dft_q(F, n, -1);
    int rc = 0;
    for (int k = 0; k < n; k++) {
        cq w = F[k];
        w.re /= n; w.im /= n;
        cq tw = cq_root(-(int64_t)k, 2 * (int64_t)N);   /* zeta^-k */
        w = cq_mul(w, tw);
        f128 a = rintq(w.re * scale), b = rintq(w.im * scale);
        if (fabsq(a) > 1.0e36Q || fabsq(b) > 1.0e36Q) rc = -1;
        out[k] = (i128)a;
        out[k + n] = (i128)b;
    }
    free(F);
    return rc;
}
/* public encode of real/imag slots (double), result as int64 (must fit) */
int orc_encode(orc_ctx *c, const double *re, const double *im, int nslots, double scale, int64_t *out) {
    cq *z = calloc(c->n, sizeof(cq));
    for (int j = 0; j < nslots && j < c->n; j++) { z[j].re = re[j]; z[j].im = im ? im[j] : 0.0; }
    i128 *m = malloc(sizeof(i128) * c->N);
    int rc = encode_q(c, z, (f128)scale, m);
    for (int k = 0; k < c->N; k++) {
        if (m[k] > (i128)INT64_MAX || m[k] < -(i128)INT64_MAX) rc = -1;
        out[k] = (int64_t)m[k];
    }
    free(z); free(m);
    return rc;
}
/* decode from quad coefficients */
static void decode_q(const orc_ctx *c, const f128 *m, f128 scale, cq *z) {
    int n = c->n, N = c->N;
    cq *F = malloc(sizeof(cq) * n);
    for (int k = 0; k < n; k++) {
        cq w = {m[k], m[k + n]};
        F[k] = cq_mul(w, cq_root(k, 2 * (int64_t)N));
    }
    dft_q(F, n, +1);
    uint64_t M = 2 * (uint64_t)N, e = 1;
    for (int j = 0; j < n; j++) {
        z[j] = F[(e - 1) / 4];
        z[j].re /= scale; z[j].im /= scale;
        e = (e * 5) % M;
    }
    free(F);
}
int orc_decode_coeffs(orc_ctx *c, const int64_t *m, double scale, double *re, double *im) {
    f128 *mq = malloc(sizeof(f128) * c->N);
    cq *z = malloc(sizeof(cq) * c->n);
    for (int k = 0; k < c->N; k++) mq[k] = m[k];
    decode_q(c, mq, scale, z);
    for (int j = 0; j < c->n; j++) { re[j] = (double)z[j].re; if (im) im[j] = (double)z[j].im; }
    free(mq); free(z);
    return 0;
}
/* brute-force embedding of integer coefficients (tests, small N only) */
int orc_embed_direct(orc_ctx *c, const int64_t *m, double *re, double *im) {
    int N = c->N;
    for (int j = 0; j < c->n; j++) {
        int e = 1;
        for (int t = 0; t < j; t++) e = (e * 5) % (2 * N);
        cq acc = {0, 0};
        for (int k = 0; k < N; k++) {
            cq w = cq_root((int64_t)e * k, 2 * (int64_t)N);
            cq v = {m[k], 0};
            acc = cq_add(acc, cq_mul(v, w));
        }
        re[j] = (double)acc.re; im[j] = (double)acc.im;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* CRT: residues mod q_0..q_l -> centred integer as quad (Garner).           */
/* ------------------------------------------------------------------------ */
static void garner_digits(const orc_ctx *c, int l, const uint64_t *x, uint64_t *v) {
    /* x = v_0 + v_1 q_0 + v_2 q_0 q_1 + ..., 0 <= v_i < q_i */
    for (int i = 0; i <= l; i++) {
        uint64_t qi = c->q[i];
        /* t = (x_i - (v_0 + v_1 q_0 + ... + v_{i-1} q_0..q_{i-2})) / (q_0..q_{i-1}) mod q_i */
        uint64_t acc = 0, prod = 1;
        for (int k = 0; k < i; k++) {
            acc = addmod(acc, mulmod(v[k] % qi, prod, qi), qi);
            prod = mulmod(prod, c->q[k] % qi, qi);
        }
        uint64_t t = submod(x[i] % qi, acc, qi);
        v[i] = mulmod(t, invmod(prod, qi), qi);
    }
}
static f128 crt_centered(const orc_ctx *c, int l, const uint64_t *x) {
    uint64_t v[128], w[128], nx[128];
    garner_digits(c, l, x, v);
    for (int i = 0; i <= l; i++) nx[i] = x[i] ? c->q[i] - x[i] : 0;
    garner_digits(c, l, nx, w);
    /* compare mixed-radix numbers from the top digit */
    int neg = 0;
    for (int i = l; i >= 0; i--) {
        if (v[i] != w[i]) { neg = (w[i] < v[i]); break; }
    }
    uint64_t *d = neg ? w : v;
    f128 acc = 0;
    for (int i = l; i >= 0; i--) acc = acc * (f128)c->q[i] + (f128)d[i];
    return neg ? -acc : acc;
}

/* ------------------------------------------------------------------------ */
/* Ciphertexts                                                               */
/* ------------------------------------------------------------------------ */
static orc_ct *ct_new(const orc_ctx *c, int level, double scale) {
    orc_ct *r = malloc(sizeof(orc_ct));
    r->level = level; r->scale = scale;
    r->c = calloc((size_t)2 * (level + 1) * c->N, sizeof(uint64_t));
    return r;
}
static inline uint64_t *ct_poly(const orc_ctx *c, const orc_ct *ct, int p) {
    return ct->c + (size_t)p * (ct->level + 1) * c->N;
}
static orc_ct *ct_copy(const orc_ctx *c, const orc_ct *a) {
    orc_ct *r = ct_new(c, a->level, a->scale);
    memcpy(r->c, a->c, sizeof(uint64_t) * 2 * (a->level + 1) * c->N);
    return r;
}
void orc_ct_free(orc_ct *ct) { if (ct) { free(ct->c); free(ct); } }
int orc_ct_level(const orc_ct *ct) { return ct->level; }
double orc_ct_scale(const orc_ct *ct) { return ct->scale; }
int orc_ct_export(orc_ctx *c, const orc_ct *ct, uint64_t *out) {
    memcpy(out, ct->c, sizeof(uint64_t) * 2 * (ct->level + 1) * c->N);
    return 0;
}
orc_ct *orc_ct_import(orc_ctx *c, const uint64_t *data, int level, double scale) {
    if (level < 0 || level > c->L) { set_err("level"); return NULL; }
    orc_ct *r = ct_new(c, level, scale);
    memcpy(r->c, data, sizeof(uint64_t) * 2 * (level + 1) * c->N);
    return r;
}

/*
 * Public-key encryption at level l:
 *   v ternary (dense), e0, e1 Gaussian, m = encode(x, scale)
 *   ct0 = v*pk0 + e0 + m,  ct1 = v*pk1 + e1   (mod q_0..q_l, NTT domain)
 */
orc_ct *orc_encrypt(orc_ctx *c, const double *x, int nslots, int level, double scale, uint64_t seed) {
    if (!c->have_sk) { set_err("no keys"); return NULL; }
    if (level < 0 || level > c->L) { set_err("level"); return NULL; }
    size_t N = c->N;
    int nq = level + 1;
    int64_t *m = malloc(sizeof(int64_t) * N);
    if (orc_encode(c, x, NULL, nslots, scale, m) != 0) { free(m); set_err("encode range"); return NULL; }
    int *idx = malloc(sizeof(int) * nq);
    for (int i = 0; i < nq; i++) idx[i] = i;
    int8_t *v = malloc(N);
    int64_t *e0 = malloc(sizeof(int64_t) * N), *e1 = malloc(sizeof(int64_t) * N);
    xof_t x0;
    xof_init(&x0, seed, mk_tag(TAG_ENC_V, 0, 0)); sample_ternary(c, &x0, v);
    xof_init(&x0, seed, mk_tag(TAG_ENC_E0, 0, 0)); sample_gauss(c, &x0, e0);
    xof_init(&x0, seed, mk_tag(TAG_ENC_E1, 0, 0)); sample_gauss(c, &x0, e1);
    for (size_t j = 0; j < N; j++) e0[j] += m[j];   /* |m| < 2^62, |e| <= 63 */
    uint64_t *vN = malloc(sizeof(uint64_t) * nq * N);
    uint64_t *a0 = malloc(sizeof(uint64_t) * nq * N);
    uint64_t *a1 = malloc(sizeof(uint64_t) * nq * N);
    small_to_ntt_i8(c, v, idx, nq, vN);
    small_to_ntt_i64(c, e0, idx, nq, a0);
    small_to_ntt_i64(c, e1, idx, nq, a1);
    orc_ct *r = ct_new(c, level, scale);
    uint64_t *pk0 = c->pk, *pk1 = c->pk + (size_t)(c->L + 1) * N;
    for (int i = 0; i < nq; i++) {
        uint64_t q = c->q[i];
        for (size_t t = 0; t < N; t++) {
            size_t o = (size_t)i * N + t;
            r->c[o] = addmod(mulmod(vN[o], pk0[o], q), a0[o], q);
            r->c[(size_t)nq * N + o] = addmod(mulmod(vN[o], pk1[o], q), a1[o], q);
        }
    }
    free(m); free(idx); free(v); free(e0); free(e1); free(vN); free(a0); free(a1);
    return r;
}

/* decrypt to the integer plaintext coefficients (centred, as double) */
static void decrypt_poly(orc_ctx *c, const orc_ct *ct, f128 *coef) {
    size_t N = c->N;
    int nq = ct->level + 1;
    uint64_t *m = malloc(sizeof(uint64_t) * nq * N);
    const uint64_t *c0 = ct_poly(c, ct, 0), *c1 = ct_poly(c, ct, 1);
    for (int i = 0; i < nq; i++) {
        uint64_t q = c->q[i];
        for (size_t t = 0; t < N; t++) {
            size_t o = (size_t)i * N + t;
            m[o] = addmod(c0[o], mulmod(c1[o], c->s_ntt[o], q), q);
        }
        ntt_inv(c, i, m + (size_t)i * N);
    }
    uint64_t x[128];
    for (size_t t = 0; t < N; t++) {
        for (int i = 0; i < nq; i++) x[i] = m[(size_t)i * N + t];
        coef[t] = crt_centered(c, ct->level, x);
    }
    free(m);
}
int orc_decrypt_coeffs(orc_ctx *c, const orc_ct *ct, double *coef) {
    f128 *q = malloc(sizeof(f128) * c->N);
    decrypt_poly(c, ct, q);
    for (int t = 0; t < c->N; t++) coef[t] = (double)q[t];
    free(q);
    return 0;
}
int orc_decrypt(orc_ctx *c, const orc_ct *ct, double *re, double *im) {
    if (!c->have_sk) { set_err("no keys"); return -1; }
    f128 *q = malloc(sizeof(f128) * c->N);
    cq *z = malloc(sizeof(cq) * c->n);
    decrypt_poly(c, ct, q);
    decode_q(c, q, (f128)ct->scale, z);
    for (int j = 0; j < c->n; j++) { re[j] = (double)z[j].re; if (im) im[j] = (double)z[j].im; }
    free(q); free(z);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Homomorphic operations                                                    */
/* ------------------------------------------------------------------------ */
/* additions require equal level and |s_a/s_b - 1| <= 2^-30; result scale s_a */
static int scales_match(double a, double b) {
    return fabs(a / b - 1.0) <= 9.313225746154785e-10;
}
orc_ct *orc_add(orc_ctx *c, const orc_ct *a, const orc_ct *b) {
    if (a->level != b->level) { set_err("level mismatch"); return NULL; }
    if (!scales_match(a->scale, b->scale)) { set_err("scale mismatch"); return NULL; }
    orc_ct *r = ct_new(c, a->level, a->scale);
    size_t N = c->N, nq = a->level + 1;
    for (int p = 0; p < 2; p++)
        for (size_t i = 0; i < nq; i++)
            for (size_t t = 0; t < N; t++) {
                size_t o = (p * nq + i) * N + t;
                r->c[o] = addmod(a->c[o], b->c[o], c->q[i]);
            }
    return r;
}
orc_ct *orc_sub(orc_ctx *c, const orc_ct *a, const orc_ct *b) {
    if (a->level != b->level) { set_err("level mismatch"); return NULL; }
    if (!scales_match(a->scale, b->scale)) { set_err("scale mismatch"); return NULL; }
    orc_ct *r = ct_new(c, a->level, a->scale);
    size_t N = c->N, nq = a->level + 1;
    for (int p = 0; p < 2; p++)
        for (size_t i = 0; i < nq; i++)
            for (size_t t = 0; t < N; t++) {
                size_t o = (p * nq + i) * N + t;
                r->c[o] = submod(a->c[o], b->c[o], c->q[i]);
            }
    return r;
}
/* multiply by the signed integer k (no level, no scale change) */
static orc_ct *mul_int64(orc_ctx *c, const orc_ct *a, int64_t k, double new_scale) {
    orc_ct *r = ct_new(c, a->level, new_scale);
    size_t N = c->N, nq = a->level + 1;
    for (size_t i = 0; i < nq; i++) {
        uint64_t q = c->q[i], kq = smod(k, q);
        for (int p = 0; p < 2; p++)
            for (size_t t = 0; t < N; t++) {
                size_t o = (p * nq + i) * N + t;
                r->c[o] = mulmod(a->c[o], kq, q);
            }
    }
    return r;
}
orc_ct *orc_mul_int(orc_ctx *c, const orc_ct *a, int64_t k) { return mul_int64(c, a, k, a->scale); }
/*
 * Mul_P by a real constant at plaintext scale s_c (no rescale):
 *   k = rint(value * s_c) (binary64 product, then rint, ties to even),
 *   ct' = k * ct,  scale' = scale * s_c.
 */
orc_ct *orc_mul_const(orc_ctx *c, const orc_ct *a, double value, double s_c) {
    double kd = rint(value * s_c);
    if (!(fabs(kd) < 4.0e18)) { set_err("constant out of range"); return NULL; }
    return mul_int64(c, a, (int64_t)kd, a->scale * s_c);
}
/* Add_P of a real constant: k = rint(value * scale) added to every NTT point of c0 */
orc_ct *orc_add_const(orc_ctx *c, const orc_ct *a, double value) {
    double kd = rint(value * a->scale);
    if (!(fabs(kd) < 4.0e18)) { set_err("constant out of range"); return NULL; }
    int64_t k = (int64_t)kd;
    orc_ct *r = ct_copy(c, a);
    size_t N = c->N, nq = a->level + 1;
    for (size_t i = 0; i < nq; i++) {
        uint64_t q = c->q[i], kq = smod(k, q);
        for (size_t t = 0; t < N; t++) r->c[i * N + t] = addmod(r->c[i * N + t], kq, q);
    }
    return r;
}
orc_ct *orc_drop_level(orc_ctx *c, const orc_ct *a, int level) {
    if (level > a->level || level < 0) { set_err("level"); return NULL; }
    orc_ct *r = ct_new(c, level, a->scale);
    size_t N = c->N;
    for (int p = 0; p < 2; p++)
        memcpy(r->c + (size_t)p * (level + 1) * N, a->c + (size_t)p * (a->level + 1) * N,
               sizeof(uint64_t) * (level + 1) * N);
    return r;
}

/*
 * Rescale: for each poly, t = iNTT_{q_l}(c_l); u = t if t <= (q_l-1)/2 else
 * t - q_l (centred lift); c'_i = (c_i - NTT_{q_i}(u mod q_i)) * q_l^{-1} mod q_i.
 * This equals round(c / q_l) coefficient-wise.  scale' = scale / q_l.
 */
orc_ct *orc_rescale(orc_ctx *c, const orc_ct *a) {
    int l = a->level;
    if (l < 1) { set_err("level"); return NULL; }
    size_t N = c->N;
    uint64_t ql = c->q[l];
    orc_ct *r = ct_new(c, l - 1, a->scale / (double)ql);
    uint64_t *t = malloc(sizeof(uint64_t) * N), *u = malloc(sizeof(uint64_t) * N);
    for (int p = 0; p < 2; p++) {
        const uint64_t *src = ct_poly(c, a, p);
        memcpy(t, src + (size_t)l * N, sizeof(uint64_t) * N);
        ntt_inv(c, l, t);
        for (int i = 0; i < l; i++) {
            uint64_t q = c->q[i];
            for (size_t k = 0; k < N; k++) {
                if (t[k] <= (ql - 1) / 2) u[k] = t[k] % q;
                else u[k] = submod(t[k] % q, ql % q, q);
            }
            ntt_fwd(c, i, u);
            uint64_t inv = invmod(ql % q, q);
            uint64_t *dst = r->c + ((size_t)p * l + i) * N;
            for (size_t k = 0; k < N; k++)
                dst[k] = mulmod(submod(src[(size_t)i * N + k], u[k], q), inv, q);
        }
    }
    free(t); free(u);
    return r;
}

/*
 * Hybrid key switch of d (NTT form, level l) with key ek.
 * Outputs (o0, o1) mod q_0..q_l (NTT form) such that
 * o0 + o1*s ~= d*s' (error small).
 *   1. d~ = iNTT(d)
 *   2. digits j = 0..beta-1, D_j = primes [jα, min((j+1)α, l+1))
 *      ModUp: for prime r outside D_j (Q_l and P):
 *        x_r = sum_{i in D_j} [d~_i * (Dhat_i)^{-1}]_{q_i} * (Dhat_i mod r)  mod r,
 *        Dhat_i = prod_{k in D_j, k != i} q_k;  then NTT_r.
 *      for r in D_j: x_r = d_r (NTT form).
 *   3. acc_b = sum_j x_j * ek_j[b]   (b = 0,1) over Q_l and P.
 *   4. ModDown: y = iNTT_P(acc_b|P); z_i = NTT_{q_i}( sum_k [y_k * Phat_k^{-1}]_{p_k}
 *      * (Phat_k mod q_i) );  o_b,i = (acc_b,i - z_i) * P^{-1} mod q_i.
 */
/* ModUp of d (NTT form, level l): for each digit j the extended
 * representation X_j[e] over Q_l and P (e = 0..ne-1), NTT form:
 * d's own limb for e in digit j, the base conversion of the digit otherwise.
 * Returns X laid out [beta][ne][N]. */
static uint64_t *modup(orc_ctx *c, int l, const uint64_t *d) {
    size_t N = c->N;
    int K = c->K, L = c->L;
    int nq = l + 1, ne = nq + K;
    int beta = (nq + c->alpha - 1) / c->alpha;
    int *ext = malloc(sizeof(int) * ne);
    for (int i = 0; i < nq; i++) ext[i] = i;
    for (int k = 0; k < K; k++) ext[nq + k] = L + 1 + k;
    uint64_t *dc = malloc(sizeof(uint64_t) * nq * N);
    memcpy(dc, d, sizeof(uint64_t) * nq * N);
    for (int i = 0; i < nq; i++) ntt_inv(c, i, dc + (size_t)i * N);
    uint64_t *X = malloc(sizeof(uint64_t) * (size_t)beta * ne * N);
    for (int j = 0; j < beta; j++) {
        int lo = j * c->alpha, hi = lo + c->alpha;
        if (hi > nq) hi = nq;
        int dn = hi - lo;
        /* [d~_i * Dhat_i^{-1}]_{q_i} */
        uint64_t *y = malloc(sizeof(uint64_t) * dn * N);
        for (int ii = 0; ii < dn; ii++) {
            int i = lo + ii;
            uint64_t qi = c->q[i], dh = 1;
            for (int kk = lo; kk < hi; kk++) if (kk != i) dh = mulmod(dh, c->q[kk] % qi, qi);
            uint64_t dhinv = invmod(dh, qi);
            for (size_t t = 0; t < N; t++) y[(size_t)ii * N + t] = mulmod(dc[(size_t)i * N + t], dhinv, qi);
        }
        for (int e = 0; e < ne; e++) {
            int pi = ext[e];
            uint64_t r = c->q[pi];
            uint64_t *x = X + ((size_t)j * ne + e) * N;
            if (e >= lo && e < hi) {
                memcpy(x, d + (size_t)e * N, sizeof(uint64_t) * N);
            } else {
                memset(x, 0, sizeof(uint64_t) * N);
                for (int ii = 0; ii < dn; ii++) {
                    int i = lo + ii;
                    uint64_t dh = 1;
                    for (int kk = lo; kk < hi; kk++) if (kk != i) dh = mulmod(dh, c->q[kk] % r, r);
                    for (size_t t = 0; t < N; t++)
                        x[t] = addmod(x[t], mulmod(y[(size_t)ii * N + t] % r, dh, r), r);
                }
                ntt_fwd(c, pi, x);
            }
        }
        free(y);
    }
    free(ext); free(dc);
    return X;
}

/* Inner product of the digits X (optionally read through the automorphism's
 * NTT-domain index map: X_j[e][perm[t]]) with the key, then ModDown by P. */
/* inner product of the digits with the key: acc_b = sum_j X_j * ek_j[b] over
 * Q_l and P (b = 0, 1), laid out [2][ne][N] */
static uint64_t *ks_inner(orc_ctx *c, int l, const uint64_t *X, const int *perm, const evk_t *ek) {
    size_t N = c->N;
    int K = c->K, L = c->L;
    int nq = l + 1, ne = nq + K;
    int beta = (nq + c->alpha - 1) / c->alpha;
    uint64_t *acc = calloc((size_t)2 * ne * N, sizeof(uint64_t));
    uint64_t *x = malloc(sizeof(uint64_t) * N);
    for (int j = 0; j < beta; j++)
        for (int e = 0; e < ne; e++) {
            int pi = e < nq ? e : L + 1 + (e - nq);
            uint64_t r = c->q[pi];
            const uint64_t *xs = X + ((size_t)j * ne + e) * N;
            for (size_t t = 0; t < N; t++) x[t] = perm ? xs[perm[t]] : xs[t];
            for (int b = 0; b < 2; b++) {
                const uint64_t *kl = ek->k + (((size_t)j * 2 + b) * c->np + pi) * N;
                uint64_t *ac = acc + ((size_t)b * ne + e) * N;
                for (size_t t = 0; t < N; t++) ac[t] = addmod(ac[t], mulmod(x[t], kl[t], r), r);
            }
        }
    free(x);
    return acc;
}

static void ks_finish(orc_ctx *c, int l, const uint64_t *X, const int *perm, const evk_t *ek, uint64_t *o0,
                      uint64_t *o1) {
    size_t N = c->N;
    int K = c->K, L = c->L;
    int nq = l + 1, ne = nq + K;
    uint64_t *acc = ks_inner(c, l, X, perm, ek);
    uint64_t *x = malloc(sizeof(uint64_t) * N);
    uint64_t *tmp = malloc(sizeof(uint64_t) * N);
    /* ModDown */
    for (int b = 0; b < 2; b++) {
        uint64_t *ac = acc + (size_t)b * ne * N;
        uint64_t *yk = malloc(sizeof(uint64_t) * K * N);
        for (int k = 0; k < K; k++) {
            int pi = L + 1 + k;
            uint64_t p = c->q[pi], ph = 1;
            memcpy(tmp, ac + (size_t)(nq + k) * N, sizeof(uint64_t) * N);
            ntt_inv(c, pi, tmp);
            for (int kk = 0; kk < K; kk++) if (kk != k) ph = mulmod(ph, c->q[L + 1 + kk] % p, p);
            uint64_t phinv = invmod(ph, p);
            for (size_t t = 0; t < N; t++) yk[(size_t)k * N + t] = mulmod(tmp[t], phinv, p);
        }
        uint64_t *o = b == 0 ? o0 : o1;
        for (int i = 0; i < nq; i++) {
            uint64_t q = c->q[i];
            memset(x, 0, sizeof(uint64_t) * N);
            uint64_t Pm = 1;
            for (int k = 0; k < K; k++) {
                uint64_t ph = 1;
                for (int kk = 0; kk < K; kk++) if (kk != k) ph = mulmod(ph, c->q[L + 1 + kk] % q, q);
                for (size_t t = 0; t < N; t++)
                    x[t] = addmod(x[t], mulmod(yk[(size_t)k * N + t] % q, ph, q), q);
                Pm = mulmod(Pm, c->q[L + 1 + k] % q, q);
            }
            ntt_fwd(c, i, x);
            uint64_t Pinv = invmod(Pm, q);
            for (size_t t = 0; t < N; t++)
                o[(size_t)i * N + t] = mulmod(submod(ac[(size_t)i * N + t], x[t], q), Pinv, q);
        }
        free(yk);
    }
    free(acc); free(x); free(tmp);
}

static void keyswitch(orc_ctx *c, int l, const uint64_t *d, const evk_t *ek, uint64_t *o0, uint64_t *o1) {
    uint64_t *X = modup(c, l, d);
    ks_finish(c, l, X, NULL, ek, o0, o1);
    free(X);
}
/* exported for tests: key switch of a raw polynomial with the relin key (-1) or rotation key */
int orc_keyswitch(orc_ctx *c, int which, int level, const uint64_t *d, uint64_t *o0, uint64_t *o1) {
    const evk_t *ek = which < 0 ? &c->relin : &c->rot[which];
    keyswitch(c, level, d, ek, o0, o1);
    return 0;
}

/*
 * Mul_C with relinearisation (no rescale):
 *   d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1;  (k0, k1) = KS(d2, relin)
 *   out = (d0 + k0, d1 + k1),  scale = s_a * s_b.
 */
orc_ct *orc_hmult(orc_ctx *c, const orc_ct *a, const orc_ct *b) {
    if (a->level != b->level) { set_err("level mismatch"); return NULL; }
    if (!c->have_sk) { set_err("no keys"); return NULL; }
    int l = a->level;
    size_t N = c->N, nq = l + 1;
    orc_ct *r = ct_new(c, l, a->scale * b->scale);
    uint64_t *d2 = malloc(sizeof(uint64_t) * nq * N);
    uint64_t *k0 = malloc(sizeof(uint64_t) * nq * N), *k1 = malloc(sizeof(uint64_t) * nq * N);
    const uint64_t *a0 = ct_poly(c, a, 0), *a1 = ct_poly(c, a, 1);
    const uint64_t *b0 = ct_poly(c, b, 0), *b1 = ct_poly(c, b, 1);
    uint64_t *r0 = ct_poly(c, r, 0), *r1 = ct_poly(c, r, 1);
    for (size_t i = 0; i < nq; i++) {
        uint64_t q = c->q[i];
        for (size_t t = 0; t < N; t++) {
            size_t o = i * N + t;
            r0[o] = mulmod(a0[o], b0[o], q);
            r1[o] = addmod(mulmod(a0[o], b1[o], q), mulmod(a1[o], b0[o], q), q);
            d2[o] = mulmod(a1[o], b1[o], q);
        }
    }
    keyswitch(c, l, d2, &c->relin, k0, k1);
    for (size_t i = 0; i < nq; i++)
        for (size_t t = 0; t < N; t++) {
            size_t o = i * N + t;
            r0[o] = addmod(r0[o], k0[o], c->q[i]);
            r1[o] = addmod(r1[o], k1[o], c->q[i]);
        }
    free(d2); free(k0); free(k1);
    return r;
}

static int find_rot(const orc_ctx *c, int g) {
    for (int i = 0; i < c->nrot; i++) if (c->rot[i].galois == g) return i;
    return -1;
}
/* automorphism X -> X^g then key switch back to s */
orc_ct *orc_automorphism(orc_ctx *c, const orc_ct *a, int g) {
    int ri = find_rot(c, g);
    if (ri < 0) { set_err("missing galois key"); return NULL; }
    int l = a->level;
    size_t N = c->N, nq = l + 1;
    int *perm = malloc(sizeof(int) * N);
    automorph_idx(c, g, perm);
    orc_ct *r = ct_new(c, l, a->scale);
    uint64_t *s0 = malloc(sizeof(uint64_t) * nq * N), *s1 = malloc(sizeof(uint64_t) * nq * N);
    const uint64_t *a0 = ct_poly(c, a, 0), *a1 = ct_poly(c, a, 1);
    for (size_t i = 0; i < nq; i++)
        for (size_t t = 0; t < N; t++) {
            s0[i * N + t] = a0[i * N + perm[t]];
            s1[i * N + t] = a1[i * N + perm[t]];
        }
    uint64_t *r0 = ct_poly(c, r, 0), *r1 = ct_poly(c, r, 1);
    keyswitch(c, l, s1, &c->rot[ri], r0, r1);
    for (size_t i = 0; i < nq; i++)
        for (size_t t = 0; t < N; t++)
            r0[i * N + t] = addmod(r0[i * N + t], s0[i * N + t], c->q[i]);
    free(perm); free(s0); free(s1);
    return r;
}
/* galois element of a left rotation by k slots: 5^k mod 2N */
int orc_galois_rot(orc_ctx *c, int k) {
    int n = c->n, M = 2 * c->N;
    k %= n; if (k < 0) k += n;
    int64_t g = 1;
    for (int t = 0; t < k; t++) g = (g * 5) % M;
    return (int)g;
}
orc_ct *orc_rotate(orc_ctx *c, const orc_ct *a, int k) {
    int g = orc_galois_rot(c, k);
    if (g == 1) return ct_copy(c, a);
    return orc_automorphism(c, a, g);
}
orc_ct *orc_conjugate(orc_ctx *c, const orc_ct *a) { return orc_automorphism(c, a, 2 * c->N - 1); }

/*
 * Hoisted rotations (Halevi-Shoup): the ModUp of c1 is computed once and
 * every rotation applies its automorphism to the extended digits (an index
 * map in the NTT domain, identical for every prime), then the inner product
 * with its key and ModDown; c0 is permuted and added.  Same result as a key
 * switch of the rotated c1 up to the base conversion's overflow term, so the
 * bits differ from orc_rotate; the slot values agree within noise.
 * steps[i] = 0 gives a copy.
 */
int orc_rotate_hoisted(orc_ctx *c, const orc_ct *a, const int *steps, int n, orc_ct **outs) {
    int l = a->level;
    size_t N = c->N, nq = l + 1;
    for (int i = 0; i < n; i++) outs[i] = NULL;
    uint64_t *X = NULL;
    int *perm = malloc(sizeof(int) * N);
    for (int i = 0; i < n; i++) {
        int g = orc_galois_rot(c, steps[i]);
        if (g == 1) { outs[i] = ct_copy(c, a); continue; }
        int ri = find_rot(c, g);
        if (ri < 0) {
            set_err("missing galois key");
            for (int k = 0; k < i; k++) { orc_ct_free(outs[k]); outs[k] = NULL; }
            free(X); free(perm);
            return -1;
        }
        if (!X) X = modup(c, l, ct_poly(c, a, 1));
        automorph_idx(c, g, perm);
        orc_ct *r = ct_new(c, l, a->scale);
        uint64_t *r0 = ct_poly(c, r, 0), *r1 = ct_poly(c, r, 1);
        ks_finish(c, l, X, perm, &c->rot[ri], r0, r1);
        const uint64_t *a0 = ct_poly(c, a, 0);
        for (size_t li = 0; li < nq; li++)
            for (size_t t = 0; t < N; t++)
                r0[li * N + t] = addmod(r0[li * N + t], a0[li * N + perm[t]], c->q[li]);
        outs[i] = r;
    }
    free(X); free(perm);
    return 0;
}

/*
 * Bring a ciphertext to level `target` (< its level) carrying the canonical
 * scale S_target:  drop to target+1, Mul_P by 1.0 at
 *   s_c = (S_target * q_{target+1}) / scale,
 * then rescale.  Same level: returned unchanged (copy).
 */
orc_ct *orc_level_to(orc_ctx *c, const orc_ct *a, int target) {
    if (target == a->level) return ct_copy(c, a);
    if (target > a->level || target < 0) { set_err("level"); return NULL; }
    orc_ct *d = orc_drop_level(c, a, target + 1);
    double sc = (c->ladder[target] * (double)c->q[target + 1]) / a->scale;
    orc_ct *m = orc_mul_const(c, d, 1.0, sc);
    orc_ct_free(d);
    if (!m) return NULL;
    orc_ct *r = orc_rescale(c, m);
    orc_ct_free(m);
    return r;
}
/* Mul_P by value landing on the canonical scale one level down:
 *   s_c = (S_{l-1} * q_l) / scale, then rescale */
static orc_ct *mul_const_down(orc_ctx *c, const orc_ct *a, double value) {
    int l = a->level;
    double sc = (c->ladder[l - 1] * (double)c->q[l]) / a->scale;
    orc_ct *m = orc_mul_const(c, a, value, sc);
    if (!m) return NULL;
    orc_ct *r = orc_rescale(c, m);
    orc_ct_free(m);
    return r;
}
orc_ct *orc_mul_const_down(orc_ctx *c, const orc_ct *a, double value) {
    if (a->level < 1) { set_err("level"); return NULL; }
    return mul_const_down(c, a, value);
}
/*
 * ModDown by P q_l of t_b = acc_b + P d_b (b = 0, 1): acc over Q_l and P
 * ([2][ne][N], NTT form), d over Q_l ([2][nq][N]); D = {q_l, p_0..p_{K-1}}:
 *   o_b,i = (acc_b,i - Conv_D(t_b)_i) (P q_l)^{-1} + d_b,i q_l^{-1}  mod q_i,  i < l,
 *   Conv_D(t)_i = NTT_{q_i}( sum_{d in D} [iNTT_d(t_d) (D/d)^{-1}]_d (D/d mod q_i) ).
 * Returns the ciphertext at level l - 1 with the given scale.
 */
static orc_ct *moddown_rescale(orc_ctx *c, int l, const uint64_t *acc, const uint64_t *d, double scale) {
    size_t N = c->N;
    int K = c->K, L = c->L, nq = l + 1, ne = nq + K;
    /* D as prime indices: q_l, then the special primes */
    int nd = K + 1;
    int *dp = malloc(sizeof(int) * nd);
    dp[0] = l;
    for (int k = 0; k < K; k++) dp[1 + k] = L + 1 + k;
    orc_ct *r = ct_new(c, l - 1, scale);
    uint64_t *yd = malloc(sizeof(uint64_t) * nd * N), *x = malloc(sizeof(uint64_t) * N);
    for (int bb = 0; bb < 2; bb++) {
        const uint64_t *ac = acc + (size_t)bb * ne * N, *db = d + (size_t)bb * nq * N;
        /* t on D, coefficient form, times (D/d)^{-1} mod d */
        for (int jd = 0; jd < nd; jd++) {
            int pi = dp[jd];
            uint64_t p = c->q[pi], dh = 1;
            uint64_t *y = yd + (size_t)jd * N;
            if (jd == 0) {   /* q_l: acc + P d (P mod q_l) */
                uint64_t Pm = 1;
                for (int k = 0; k < K; k++) Pm = mulmod(Pm, c->q[L + 1 + k] % p, p);
                for (size_t t = 0; t < N; t++)
                    y[t] = addmod(ac[(size_t)l * N + t], mulmod(db[(size_t)l * N + t], Pm, p), p);
            } else {         /* special prime: acc (P d = 0 there) */
                memcpy(y, ac + (size_t)(nq + jd - 1) * N, sizeof(uint64_t) * N);
            }
            ntt_inv(c, pi, y);
            for (int kk = 0; kk < nd; kk++) if (kk != jd) dh = mulmod(dh, c->q[dp[kk]] % p, p);
            uint64_t dhinv = invmod(dh, p);
            for (size_t t = 0; t < N; t++) y[t] = mulmod(y[t], dhinv, p);
        }
        uint64_t *o = r->c + (size_t)bb * l * N;
        for (int i = 0; i < l; i++) {
            uint64_t q = c->q[i];
            memset(x, 0, sizeof(uint64_t) * N);
            uint64_t Dm = 1;
            for (int jd = 0; jd < nd; jd++) {
                uint64_t dh = 1;
                for (int kk = 0; kk < nd; kk++) if (kk != jd) dh = mulmod(dh, c->q[dp[kk]] % q, q);
                for (size_t t = 0; t < N; t++) x[t] = addmod(x[t], mulmod(yd[(size_t)jd * N + t] % q, dh, q), q);
                Dm = mulmod(Dm, c->q[dp[jd]] % q, q);
            }
            ntt_fwd(c, i, x);
            uint64_t Dinv = invmod(Dm, q), qlinv = invmod(c->q[l] % q, q);
            for (size_t t = 0; t < N; t++) {
                size_t e = (size_t)i * N + t;
                o[e] = addmod(mulmod(submod(ac[e], x[t], q), Dinv, q), mulmod(db[e], qlinv, q), q);
            }
        }
    }
    free(yd); free(x); free(dp);
    return r;
}

/*
 * Mul_C, relinearise and rescale, with the rescale merged into the key
 * switch's ModDown (one division by P q_l instead of a division by P, then a
 * rounding division by q_l).  With the tensor (d0, d1, d2), the key switch's
 * accumulator acc_b over Q_l and P (inner product of ModUp(d2) with the
 * relinearisation key), t_b = acc_b + P d_b (d_b over Q_l only; zero mod P)
 * and D = {q_l, p_0..p_{K-1}}:
 *   o_b,i = (t_b,i - Conv_D(t_b)_i) (P q_l)^{-1}  mod q_i,  i < l,
 *   Conv_D(t)_i = NTT_{q_i}( sum_{d in D} [iNTT_d(t_d) (D/d)^{-1}]_d (D/d mod q_i) ),
 * computed as (acc_b,i - Conv_D(t_b)_i) (P q_l)^{-1} + d_b,i q_l^{-1}.  This is
 * t / (P q_l) up to the approximate conversion's small overshoot (as in
 * ModDown); scale' = s_a s_b / q_l, level l - 1.
 */
static orc_ct *mult_rs(orc_ctx *c, const orc_ct *a, const orc_ct *b) {
    if (a->level != b->level) { set_err("level mismatch"); return NULL; }
    if (!c->have_sk) { set_err("no keys"); return NULL; }
    int l = a->level;
    if (l < 1) { set_err("level"); return NULL; }
    size_t N = c->N;
    int K = c->K, L = c->L, nq = l + 1, ne = nq + K;
    uint64_t *d = malloc(sizeof(uint64_t) * 2 * nq * N), *d2 = malloc(sizeof(uint64_t) * nq * N);
    const uint64_t *a0 = ct_poly(c, a, 0), *a1 = ct_poly(c, a, 1);
    const uint64_t *b0 = ct_poly(c, b, 0), *b1 = ct_poly(c, b, 1);
    for (int i = 0; i < nq; i++) {
        uint64_t q = c->q[i];
        for (size_t t = 0; t < N; t++) {
            size_t o = (size_t)i * N + t;
            d[o] = mulmod(a0[o], b0[o], q);
            d[(size_t)nq * N + o] = addmod(mulmod(a0[o], b1[o], q), mulmod(a1[o], b0[o], q), q);
            d2[o] = mulmod(a1[o], b1[o], q);
        }
    }
    uint64_t *X = modup(c, l, d2);
    uint64_t *acc = ks_inner(c, l, X, NULL, &c->relin);
    free(X); free(d2);
    orc_ct *r = moddown_rescale(c, l, acc, d, a->scale * b->scale / (double)c->q[l]);
    free(acc); free(d);
    return r;
}
/* exported for tests: the merged relinearise-and-rescale product */
orc_ct *orc_mult_rs(orc_ctx *c, const orc_ct *a, const orc_ct *b) { return mult_rs(c, a, b); }

/* aligned product: both operands brought to the lower of their levels */
static orc_ct *mult_aligned(orc_ctx *c, const orc_ct *a, const orc_ct *b) {
    int l = a->level < b->level ? a->level : b->level;
    if (l < 1) { set_err("level"); return NULL; }
    orc_ct *x = orc_level_to(c, a, l), *y = orc_level_to(c, b, l);
    orc_ct *r = mult_rs(c, x, y);
    orc_ct_free(x); orc_ct_free(y);
    return r;
}
/* aligned sum / difference */
static orc_ct *addsub_aligned(orc_ctx *c, const orc_ct *a, const orc_ct *b, int sub) {
    int l = a->level < b->level ? a->level : b->level;
    orc_ct *x = orc_level_to(c, a, l), *y = orc_level_to(c, b, l);
    orc_ct *r = sub ? orc_sub(c, x, y) : orc_add(c, x, y);
    orc_ct_free(x); orc_ct_free(y);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev interpolant (paper §2.3: the initial value y_0 is a Chebyshev   */
/* approximation of 1/sqrt).  Interpolation at the n = d+1 first-kind nodes: */
/*   theta_j = pi (j + 1/2) / n,  x_j = (a+b)/2 + (b-a)/2 cos(theta_j)        */
/*   c_k = (2/n) sum_j f(x_j) cos(k theta_j),   c_0 halved.                  */
/* Computed in quad, rounded once to binary64.                               */
/* ------------------------------------------------------------------------ */
typedef f128 (*qfun)(f128 x, const double *par);
static f128 f_invsqrt(f128 x, const double *par) { (void)par; return 1 / sqrtq(x); }
/* cos(2*pi*(K*x - 1/4) / 2^r):  par[0] = K, par[1] = 2^r */
static f128 f_cosmod(f128 x, const double *par) {
    return cosq(2 * M_PIq * ((f128)par[0] * x - 0.25Q) / (f128)par[1]);
}
static void cheb_interp(int d, double a, double b, qfun f, const double *par, double *out) {
    int n = d + 1;
    f128 A = a, B = b;
    f128 *fx = malloc(sizeof(f128) * n);
    for (int j = 0; j < n; j++) {
        f128 th = M_PIq * ((f128)j + 0.5Q) / (f128)n;
        f128 x = (A + B) / 2 + (B - A) / 2 * cosq(th);
        fx[j] = f(x, par);
    }
    for (int k = 0; k <= d; k++) {
        f128 s = 0;
        for (int j = 0; j < n; j++) {
            f128 th = M_PIq * ((f128)j + 0.5Q) / (f128)n;
            s += fx[j] * cosq((f128)k * th);
        }
        s = s * 2 / (f128)n;
        if (k == 0) s /= 2;
        out[k] = (double)s;
    }
    free(fx);
}
int orc_cheb_coeffs_invsqrt(int d, double a, double b, double *out) {
    if (d < 1 || !(a > 0) || !(b > a)) return -1;
    cheb_interp(d, a, b, f_invsqrt, NULL, out);
    return 0;
}
int orc_cheb_coeffs_cosmod(int d, double K, double two_r, double *out) {
    double par[2] = {K, two_r};
    cheb_interp(d, -1.0, 1.0, f_cosmod, par, out);
    return 0;
}

/*
 * Chebyshev-basis evaluation by baby-step / giant-step (a reading: the paper
 * names only "ChebyshevApprox"; it fixes the depth, §4.3: a degree-2^{d_e}-2
 * polynomial consumes d_e levels, §3: degree 2^9-2 has depth 9).  For
 * degree d:
 *   m = bit length of d, b = ceil(m/2);
 *   baby powers T_1..T_{2^b - 1}, giant powers T_{2^b}, T_{2^{b+1}}, ..., T_{2^{m-1}}
 *   T_{2k} = 2 T_k^2 - 1,  T_{2k+1} = 2 T_{k+1} T_k - T_1   (k >= 1), products
 *   taken on operands brought to the lower level (level_to) and rescaled;
 *   T_i then sits ceil(log2 i) levels below t.
 *   eval(p, k, D) for deg p < 2^k, with a budget of D >= k levels below t:
 *     leaf if k <= b and deg p <= 2^{D-1} (every T_i it combines is at most
 *       D-1 levels down, and the combination takes one level): baby linear
 *       combination;
 *     else M = 2^{k-1}; if deg < M recurse with (k-1, D); else split
 *     p = q*T_M + r with q_0 = c_M, q_j = 2 c_{M+j} (j >= 1),
 *     r_i = c_i (i < M) then r_{M-j} = c_{M-j} - c_{M+j} (j >= 1);
 *     result = level-aligned (eval(q, k-1, D-1) * T_M) + eval(r, k-1, D).
 *   The whole polynomial is eval(p, m, m): only the leading quotient chain
 *   has D = k, and it is split below the baby-step height down to degree 1
 *   (its products by T_{2^j}, j < b, replace the baby combination that
 *   would cost one level more), so the evaluation takes exactly m levels.
 *   baby combination of c_0..c_t: terms i >= 1 with c_i != 0 (if
 *   none, i = 1 with coefficient 0.0); l_min = lowest level of those T_i;
 *   each T_i is dropped to l_min and multiplied by c_i at
 *   s_c = (S_{l_min - 1} * q_{l_min}) / scale(T_i); the products are summed
 *   in increasing i, rescaled once, and c_0 is added with Add_P.
 * The variable t = alpha*x + beta, alpha = 2/(b-a), beta = -(a+b)/(b-a), is
 * formed first with one Mul_P (landing on the canonical scale) and one Add_P;
 * for [a,b] = [-1,1] the input is used as t directly.
 */
typedef struct { orc_ct **T; int maxT; } powtab;

static orc_ct *pw_get(orc_ctx *c, powtab *pt, int i);
static orc_ct *pw_compute(orc_ctx *c, powtab *pt, int i) {
    /* i >= 2 */
    orc_ct *r;
    if ((i & 1) == 0) {
        orc_ct *h = pw_get(c, pt, i / 2);
        orc_ct *sq = mult_rs(c, h, h);
        if (!sq) return NULL;
        orc_ct *d = orc_mul_int(c, sq, 2);
        orc_ct_free(sq);
        r = orc_add_const(c, d, -1.0);
        orc_ct_free(d);
    } else {
        orc_ct *a = pw_get(c, pt, (i + 1) / 2), *b = pw_get(c, pt, (i - 1) / 2);
        if (!a || !b) return NULL;
        orc_ct *p = mult_aligned(c, a, b);
        if (!p) return NULL;
        orc_ct *d = orc_mul_int(c, p, 2);
        orc_ct_free(p);
        r = addsub_aligned(c, d, pt->T[1], 1);
        orc_ct_free(d);
    }
    return r;
}
static orc_ct *pw_get(orc_ctx *c, powtab *pt, int i) {
    if (pt->T[i]) return pt->T[i];
    pt->T[i] = pw_compute(c, pt, i);
    return pt->T[i];
}

static orc_ct *baby_combo(orc_ctx *c, powtab *pt, const double *cf, int deg) {
    int lmin = 1 << 30, any = 0;
    for (int i = 1; i <= deg; i++) if (cf[i] != 0.0) { any = 1; if (pt->T[i]->level < lmin) lmin = pt->T[i]->level; }
    if (!any) lmin = pt->T[1]->level;
    if (lmin < 1) { set_err("level"); return NULL; }
    orc_ct *acc = NULL;
    for (int i = 1; i <= deg || (!any && i == 1); i++) {
        double ci = any ? cf[i] : 0.0;
        if (any && ci == 0.0) continue;
        orc_ct *d = orc_drop_level(c, pt->T[i], lmin);
        double sc = (c->ladder[lmin - 1] * (double)c->q[lmin]) / pt->T[i]->scale;
        orc_ct *m = orc_mul_const(c, d, ci, sc);
        orc_ct_free(d);
        if (!m) { orc_ct_free(acc); return NULL; }
        if (!acc) acc = m;
        else {
            orc_ct *s = orc_add(c, acc, m);
            orc_ct_free(acc); orc_ct_free(m);
            if (!s) return NULL;
            acc = s;
        }
        if (!any) break;
    }
    orc_ct *r = orc_rescale(c, acc);
    orc_ct_free(acc);
    if (!r) return NULL;
    orc_ct *r2 = orc_add_const(c, r, cf[0]);
    orc_ct_free(r);
    return r2;
}
static orc_ct *cheb_rec(orc_ctx *c, powtab *pt, const double *cf, int deg, int k, int D, int b) {
    if (k <= b && deg <= (1 << (D - 1))) return baby_combo(c, pt, cf, deg);
    int M = 1 << (k - 1);
    if (deg < M) return cheb_rec(c, pt, cf, deg, k - 1, D, b);
    int dq = deg - M;
    double *qc = malloc(sizeof(double) * (dq + 1));
    double *rc = malloc(sizeof(double) * M);
    qc[0] = cf[M];
    for (int j = 1; j <= dq; j++) qc[j] = 2.0 * cf[M + j];
    for (int i = 0; i < M; i++) rc[i] = cf[i];
    for (int j = 1; j <= dq; j++) rc[M - j] = cf[M - j] - cf[M + j];
    orc_ct *Q = cheb_rec(c, pt, qc, dq, k - 1, D - 1, b);
    orc_ct *R = Q ? cheb_rec(c, pt, rc, M - 1, k - 1, D, b) : NULL;
    free(qc); free(rc);
    if (!Q || !R) { orc_ct_free(Q); orc_ct_free(R); return NULL; }
    orc_ct *TM = pw_get(c, pt, M);
    orc_ct *P = TM ? mult_aligned(c, Q, TM) : NULL;
    orc_ct_free(Q);
    if (!P) { orc_ct_free(R); return NULL; }
    orc_ct *out = addsub_aligned(c, P, R, 0);
    orc_ct_free(P); orc_ct_free(R);
    return out;
}
static int bitlen(int d) { int m = 0; while (d >> m) m++; return m; }

orc_ct *orc_cheb_eval(orc_ctx *c, const orc_ct *x, const double *cf, int d, double a, double b) {
    if (d < 1) { set_err("degree"); return NULL; }
    orc_ct *t;
    if (a == -1.0 && b == 1.0) t = ct_copy(c, x);
    else {
        if (x->level < 1) { set_err("level"); return NULL; }
        double al = 2.0 / (b - a);
        double be = -(a + b) / (b - a);
        orc_ct *m = mul_const_down(c, x, al);
        if (!m) return NULL;
        t = orc_add_const(c, m, be);
        orc_ct_free(m);
    }
    int m = bitlen(d), bb = (m + 1) / 2;
    powtab pt;
    pt.maxT = 1 << m;
    pt.T = calloc(pt.maxT + 1, sizeof(orc_ct *));
    pt.T[1] = t;
    /* baby powers, in increasing index */
    int nb = 1 << bb;
    for (int i = 2; i < nb && i <= d; i++) if (!pw_get(c, &pt, i)) goto fail;
    /* giant powers */
    for (int k = bb; k < m; k++) if (!pw_get(c, &pt, 1 << k)) goto fail;
    {
        orc_ct *r = cheb_rec(c, &pt, cf, d, m, m, bb);
        for (int i = 1; i <= pt.maxT; i++) orc_ct_free(pt.T[i]);
        free(pt.T);
        return r;
    }
fail:
    for (int i = 1; i <= pt.maxT; i++) orc_ct_free(pt.T[i]);
    free(pt.T);
    return NULL;
}

/* ------------------------------------------------------------------------ */
/* Newton step for 1/sqrt (paper §2.2; Alg. 1 loop body):                   */
/*   tmp_a = Mul_P(y, 1.5); tmp_b = Mul_C(ct_x, y); y2 = Mul_C(y, y);        */
/*   tmp_b = Mul_C(tmp_b, y2); y' = tmp_a - tmp_b                            */
/* with ct_x = x/2.  Level placement: c = min(l_x, l_y) (needs c >= 2);      */
/*   x at level c: level_to (canonical) or, with raw_x, a plain limb drop    */
/*   that keeps x's own scale;  u = (x@c)(y@c) -> c-1;                       */
/*   v = (y@c)(y@c) -> c-1 (y aligned once, both products at one level);    */
/*   w = u*v -> c-2;                                                         */
/*   tmp_a = y dropped to c-1, Mul_P 1.5 at s_c = (scale(w) q_{c-1}) /       */
/*   scale(y), rescaled, so that it lands exactly on scale(w).               */
/* ------------------------------------------------------------------------ */
/* with the constant c15 of tmp_a (1.5 in the step of §2.2) */
static orc_ct *newton_step(orc_ctx *c, const orc_ct *y, const orc_ct *ctx_half, int raw_x, double c15) {
    int lc = y->level < ctx_half->level ? y->level : ctx_half->level;
    if (lc < 2) { set_err("level"); return NULL; }
    orc_ct *xa = raw_x ? orc_drop_level(c, ctx_half, lc) : orc_level_to(c, ctx_half, lc);
    orc_ct *ya = orc_level_to(c, y, lc);
    orc_ct *u = mult_rs(c, xa, ya);
    orc_ct *v = mult_rs(c, ya, ya);
    orc_ct_free(xa); orc_ct_free(ya);
    orc_ct *w = mult_rs(c, u, v);
    orc_ct_free(u); orc_ct_free(v);
    orc_ct *yd = orc_drop_level(c, y, lc - 1);
    double sc = (w->scale * (double)c->q[lc - 1]) / yd->scale;
    orc_ct *tm = orc_mul_const(c, yd, c15, sc);
    orc_ct_free(yd);
    orc_ct *ta = orc_rescale(c, tm);
    orc_ct_free(tm);
    orc_ct *r = orc_sub(c, ta, w);
    orc_ct_free(ta); orc_ct_free(w);
    return r;
}
orc_ct *orc_newton_step_ex(orc_ctx *c, const orc_ct *y, const orc_ct *ctx_half, int raw_x) {
    return newton_step(c, y, ctx_half, raw_x, 1.5);
}
orc_ct *orc_newton_step(orc_ctx *c, const orc_ct *y, const orc_ct *ctx_half) {
    return orc_newton_step_ex(c, y, ctx_half, 0);
}

/* ------------------------------------------------------------------------ */
/* Bootstrapping (§2.1: BTS resets a ciphertext's level to l_afterBTS; the  */
/* scheme's bootstrapping as cited there).  Written from the CKKS           */
/* bootstrapping construction: ModRaise, CoeffToSlot, EvalMod (cosine and   */
/* double angle), SlotToCoeff.                                               */
/*                                                                           */
/* Slot transform.  With n = N/2 slots at the roots zeta^(5^j) (zeta =      */
/* exp(i pi / N)), slot j of a real polynomial p is                          */
/*   z_j = sum_{k<n} w_k zeta^(5^j k),   w_k = p_k + i p_{k+n},             */
/* i.e. z = V w.  V factors as V = B_n B_{n/2} ... B_2 R, R the bit          */
/* reversal of w and B_len (len = 2^k) block diagonal with blocks of length  */
/* len, each butterfly pairing positions j and j + len/2 of its block:       */
/*   y_j = x_j + t_j x_{j+len/2},  y_{j+len/2} = x_j - t_j x_{j+len/2},      */
/*   t_j = exp(2 pi i (5^j mod 4 len) / (4 len)),  j < len/2.                */
/* CoeffToSlot applies B_n^-1, ..., B_2^-1 (output: R w, coefficients in bit  */
/* reversed order) and SlotToCoeff applies B_2, ..., B_n to R w, so R is      */
/* never evaluated.  The log2(n) stages are grouped into three groups of     */
/* floor(log2 n / 3) stages, the first (log2 n mod 3) groups, counted from   */
/* the top stage, taking one more; each group is one plaintext-matrix        */
/* product (one level), evaluated by baby-step giant-step over its nonzero   */
/* diagonals.                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kmin, kmax;  /* stages k in [kmin, kmax] (butterfly length 2^k) */
    int s;           /* offset stride 2^(kmin-1) */
    int g;           /* giant step, in units of s */
    int nm;          /* nonzero diagonals */
    int *m;          /* their offsets in units of s, ascending */
    cq **d;          /* d[t][j] = M[j][(j + m[t] s) mod n] */
} lt_group;

struct bts_plan {
    double Kp;       /* EvalMod interval: t = p/q_0 in [-Kp, Kp] */
    int r, deg;      /* double-angle steps, Chebyshev degree of the cosine */
    double *cf;
    lt_group cts[3], stc[3];   /* in application order */
    double cts_sd[3], stc_sd[3];   /* plaintext scale of each stage */
};

static void lt_free(lt_group *G) {
    for (int t = 0; t < G->nm; t++) free(G->d[t]);
    free(G->d); free(G->m);
    memset(G, 0, sizeof(*G));
}
static void bts_plan_free(struct bts_plan *b) {
    if (!b) return;
    for (int i = 0; i < 3; i++) { lt_free(&b->cts[i]); lt_free(&b->stc[i]); }
    free(b->cf);
    free(b);
}

/* the three nonzero diagonals of B_len (inv: of its inverse) at offsets
 * 0, +len/2, -len/2 (mod n); with len = n the last two offsets coincide */
static void stage_diags(int n, int k, int inv, cq *d0, cq *dp, cq *dm) {
    int len = 1 << k, h = len / 2;
    for (int j = 0; j < n; j++) {
        int jj = j % len;
        cq zero = {0, 0}, one = {1, 0};
        d0[j] = zero; dp[j] = zero; dm[j] = zero;
        if (jj < h) {
            cq t = cq_root((int64_t)powmod(5, (uint64_t)jj, 4 * (uint64_t)len), 4 * (int64_t)len);
            if (!inv) { d0[j] = one; dp[j] = t; }
            else { cq half = {0.5Q, 0}; d0[j] = half; dp[j] = half; }
        } else {
            cq t = cq_root((int64_t)powmod(5, (uint64_t)(jj - h), 4 * (uint64_t)len), 4 * (int64_t)len);
            if (!inv) { cq mt = {-t.re, -t.im}; d0[j] = mt; dm[j] = one; }
            else {
                /* 1 / (2 t) = conj(t) / 2 since |t| = 1 */
                cq ih = {t.re / 2, -t.im / 2};
                cq mih = {-ih.re, -ih.im};
                dm[j] = ih; d0[j] = mih;
            }
        }
    }
}

/* product of the stages ks[0..cnt-1] (applied in that order) in diagonal form */
static void group_build(int n, const int *ks, int cnt, int inv, f128 cmul, lt_group *G) {
    cq **cur = calloc(n, sizeof(cq *));
    cur[0] = malloc(sizeof(cq) * n);
    for (int j = 0; j < n; j++) { cur[0][j].re = cmul; cur[0][j].im = 0; }
    cq *sd[3];
    for (int i = 0; i < 3; i++) sd[i] = malloc(sizeof(cq) * n);
    G->kmin = ks[0]; G->kmax = ks[0];
    for (int t = 0; t < cnt; t++) {
        int k = ks[t], h = 1 << (k - 1);
        if (k < G->kmin) G->kmin = k;
        if (k > G->kmax) G->kmax = k;
        stage_diags(n, k, inv, sd[0], sd[1], sd[2]);
        int off[3] = {0, h % n, (n - h) % n};
        cq **nx = calloc(n, sizeof(cq *));
        for (int p = 0; p < n; p++) {
            if (!cur[p]) continue;
            for (int e = 0; e < 3; e++) {
                int o = off[e], dst = (o + p) % n;
                if (!nx[dst]) nx[dst] = calloc(n, sizeof(cq));
                for (int j = 0; j < n; j++) {
                    cq v = cq_mul(sd[e][j], cur[p][(j + o) % n]);
                    nx[dst][j] = cq_add(nx[dst][j], v);
                }
            }
        }
        for (int p = 0; p < n; p++) free(cur[p]);
        free(cur);
        cur = nx;
    }
    for (int i = 0; i < 3; i++) free(sd[i]);
    G->s = 1 << (G->kmin - 1);
    int ns = n / G->s, nk = G->kmax - G->kmin + 1;
    int wrap = ns <= (1 << nk);
    G->nm = 0;
    G->m = malloc(sizeof(int) * n);
    G->d = malloc(sizeof(cq *) * n);
    /* collect nonzero diagonals, as signed offsets m (units of s) */
    int *mm = malloc(sizeof(int) * n);
    cq **dd = malloc(sizeof(cq *) * n);
    int cntd = 0;
    for (int o = 0; o < n; o++) {
        if (!cur[o]) continue;
        int nz = 0;
        for (int j = 0; j < n && !nz; j++) nz = (cur[o][j].re != 0 || cur[o][j].im != 0);
        if (!nz) { free(cur[o]); continue; }
        int m = o / G->s;                    /* every offset is a multiple of s */
        if (!wrap && m > ns / 2) m -= ns;
        mm[cntd] = m; dd[cntd] = cur[o]; cntd++;
    }
    free(cur);
    /* ascending m */
    for (int i = 0; i < cntd; i++) {
        int best = i;
        for (int j = i + 1; j < cntd; j++) if (mm[j] < mm[best]) best = j;
        int tm = mm[i]; mm[i] = mm[best]; mm[best] = tm;
        cq *td = dd[i]; dd[i] = dd[best]; dd[best] = td;
    }
    for (int i = 0; i < cntd; i++) { G->m[i] = mm[i]; G->d[i] = dd[i]; }
    G->nm = cntd;
    free(mm); free(dd);
    int span = G->m[cntd - 1] - G->m[0] + 1, e = 0;
    while ((1 << e) < span) e++;
    G->g = 1 << ((e + 1) / 2);
}

/* content scale of a unit message at the bootstrapping input: q_0 2^-5 */
static double bts_content_scale(const orc_ctx *c) { return ldexp((double)c->q[0], -5); }

static int floordiv(int a, int b) { int q = a / b; if ((a % b) != 0 && ((a < 0) != (b < 0))) q--; return q; }

/*
 * Configure bootstrapping: EvalMod approximates cos(2 pi (Kp u - 1/4) / 2^r)
 * on u in [-1, 1] by a degree-`deg` Chebyshev interpolant (u = t / Kp,
 * t = p / q_0 the ModRaised coefficient over q_0) and applies r double-angle
 * steps cos(2a) = 2 cos(a)^2 - 1, giving sin(2 pi t).  Requires the chain's
 * SlotToCoeff and CoeffToSlot regions to have three levels each and EvalMod
 * to have cheb_depth(deg) + r levels.
 */
/* levels the Chebyshev evaluation above consumes for degree d on [-1, 1]:
 * the bit length of d (§4.3's d_e for degree 2^{d_e} - 2) */
static int cheb_depth(int d) { return bitlen(d); }
int orc_cheb_depth(int d) { return d >= 1 ? cheb_depth(d) : -1; }
int orc_bts_config(orc_ctx *c, double Kp, int r, int deg) {
    if (c->n_evm <= 0) { set_err("chain has no bootstrapping levels"); return -1; }
    if (c->n_stc != 3 || c->n_cts != 3 || c->n_evm != cheb_depth(deg) + r || Kp <= 1 || r < 0 || deg < 2) {
        set_err("bootstrapping configuration does not match the chain");
        return -1;
    }
    bts_plan_free(c->bts);
    struct bts_plan *b = calloc(1, sizeof(*b));
    b->Kp = Kp; b->r = r; b->deg = deg;
    b->cf = malloc(sizeof(double) * (deg + 1));
    orc_cheb_coeffs_cosmod(deg, Kp, ldexp(1.0, r), b->cf);
    int n = c->n, logn = c->logN - 1;
    int sizes[3], top = logn;
    for (int i = 0; i < 3; i++) sizes[i] = logn / 3 + (i < logn % 3 ? 1 : 0);
    f128 cs = (f128)c->q[0] / (2 * M_PIq * (f128)bts_content_scale(c));
    for (int i = 0; i < 3; i++) {
        int ks[32];
        /* CoeffToSlot group i: stages top, top-1, ..., applied in that order */
        for (int t = 0; t < sizes[i]; t++) ks[t] = top - t;
        group_build(n, ks, sizes[i], 1, 1.0Q, &b->cts[i]);
        /* the SlotToCoeff group with the same stages is applied at position 2-i,
         * its stages ascending; the first one applied carries q_0 / (2 pi s_0),
         * s_0 = q_0 2^-5 the input content scale of a unit message */
        int kr[32];
        for (int t = 0; t < sizes[i]; t++) kr[t] = top - sizes[i] + 1 + t;
        group_build(n, kr, sizes[i], 0, i == 2 ? cs : 1.0Q, &b->stc[2 - i]);
        top -= sizes[i];
    }
    /* plaintext scales from the nominal scale chain.  CoeffToSlot starts at
     * the ModRaise scale D = 2 q_0 Kp and ends on S_{L-3}; SlotToCoeff starts
     * at S_{l_after+3} (the EvalMod output) and ends on S_{l_after}.  With
     * f = cbrt(end / start) the stage targets are start f, start f f, end;
     * stage t at level lv has s_d = (target * q_lv) / s and leaves the
     * scale (s * s_d) / q_lv. */
    for (int pass = 0; pass < 2; pass++) {
        int lv = pass == 0 ? c->L : c->l_after + 3;
        double s = pass == 0 ? 2.0 * (double)c->q[0] * Kp : c->ladder[c->l_after + 3];
        double end = pass == 0 ? c->ladder[c->L - 3] : c->ladder[c->l_after];
        double f = cbrt(end / s);
        double tg[3];
        tg[0] = s * f;
        tg[1] = tg[0] * f;
        tg[2] = end;
        double *sd = pass == 0 ? b->cts_sd : b->stc_sd;
        for (int t = 0; t < 3; t++, lv--) {
            sd[t] = (tg[t] * (double)c->q[lv]) / s;
            s = (s * sd[t]) / (double)c->q[lv];
        }
    }
    c->bts = b;
    return 0;
}

static void lt_steps(const orc_ctx *c, const lt_group *G, int *seen, int n) {
    for (int t = 0; t < G->nm; t++) {
        int i = floordiv(G->m[t], G->g), bb = G->m[t] - G->g * i;
        int kb = (int)(((int64_t)bb * G->s) % n);
        int kg = (int)((((int64_t)G->g * i * G->s) % n + n) % n);
        if (kb) seen[kb] = 1;
        if (kg) seen[kg] = 1;
    }
    (void)c;
}
/* left-rotation amounts (in [1, n)) whose Galois keys bootstrapping uses,
 * ascending; the conjugation key (2N - 1) is needed as well */
int orc_bts_rotations(orc_ctx *c, int32_t *out, int max) {
    if (!c->bts) { set_err("bootstrapping not configured"); return -1; }
    int n = c->n, cnt = 0;
    int *seen = calloc(n, sizeof(int));
    for (int i = 0; i < 3; i++) { lt_steps(c, &c->bts->cts[i], seen, n); lt_steps(c, &c->bts->stc[i], seen, n); }
    for (int k = 1; k < n; k++)
        if (seen[k]) { if (out && cnt < max) out[cnt] = k; cnt++; }
    free(seen);
    return cnt;
}

static uint64_t i128_mod(i128 v, uint64_t q) {
    i128 r = v % (i128)q;
    if (r < 0) r += q;
    return (uint64_t)r;
}

/* baby-step giant-step product of a group matrix with the slots of x:
 *   out = sum_i rot_{g i s}( sum_b P_{i,b} * rot_{b s}(x) ),
 *   every rotation in the hoisted form (the babies share one ModUp of x),
 *   P_{i,b} = diagonal m = g i + b rotated right by g i s, encoded at
 *   scale sd;  one rescale at the end (scale (scale(x) sd) / q_l). */
static orc_ct *lt_apply(orc_ctx *c, const orc_ct *x, const lt_group *G, double sd) {
    int l = x->level, n = c->n;
    size_t N = c->N;
    if (l < 1) { set_err("level"); return NULL; }
    int g = G->g;
    /* baby steps: every used b, rotated by b s, all from one hoisted ModUp */
    orc_ct **R = calloc(g, sizeof(orc_ct *));
    int *used = calloc(g, sizeof(int)), *bsteps = malloc(sizeof(int) * g), nb = 0;
    for (int t = 0; t < G->nm; t++) {
        int i = floordiv(G->m[t], g), bb = G->m[t] - g * i;
        used[bb] = 1;
    }
    for (int bb = 0; bb < g; bb++) if (used[bb]) bsteps[nb++] = bb;
    orc_ct **Rb = calloc(g, sizeof(orc_ct *));
    int *kst = malloc(sizeof(int) * g);
    for (int t = 0; t < nb; t++) kst[t] = bsteps[t] * G->s;
    int rc = orc_rotate_hoisted(c, x, kst, nb, Rb);
    for (int t = 0; t < nb; t++) R[bsteps[t]] = Rb[t];
    free(Rb); free(kst); free(used); free(bsteps);
    if (rc != 0) { free(R); return NULL; }
    cq *v = malloc(sizeof(cq) * n);
    i128 *coef = malloc(sizeof(i128) * N);
    uint64_t *pt = malloc(sizeof(uint64_t) * N);
    /* giant steps: the rotated ones' key-switch accumulators summed over Q_l
     * and P (A), their rotated c0 and giant 0's inner sum summed over Q_l (E);
     * the output is ModDown by P q_l of A + P E (the rescale merged) */
    int K = c->K, nq = l + 1, ne = nq + K;
    uint64_t *A = calloc((size_t)2 * ne * N, sizeof(uint64_t));
    uint64_t *E = calloc((size_t)2 * nq * N, sizeof(uint64_t));
    int *perm = malloc(sizeof(int) * N);
    int nrot = 0;
    orc_ct *acc = NULL;
    int imin = floordiv(G->m[0], g), imax = floordiv(G->m[G->nm - 1], g);
    int fail = 0;
    for (int i = imin; i <= imax && !fail; i++) {
        orc_ct *inner = NULL;
        for (int t = 0; t < G->nm; t++) {
            if (floordiv(G->m[t], g) != i) continue;
            int bb = G->m[t] - g * i;
            int64_t sh = (int64_t)g * i * G->s;
            for (int j = 0; j < n; j++) {
                int64_t src = (((int64_t)j - sh) % n + n) % n;
                v[j] = G->d[t][src];
            }
            if (encode_q(c, v, (f128)sd, coef) != 0) { set_err("diagonal out of range"); fail = 1; break; }
            if (!inner) { inner = ct_new(c, l, x->scale * sd); memset(inner->c, 0, sizeof(uint64_t) * 2 * (l + 1) * N); }
            for (int li = 0; li <= l; li++) {
                uint64_t q = c->q[li];
                for (size_t k = 0; k < N; k++) pt[k] = i128_mod(coef[k], q);
                ntt_fwd(c, li, pt);
                for (int p = 0; p < 2; p++) {
                    const uint64_t *src = ct_poly(c, R[bb], p) + (size_t)li * N;
                    uint64_t *dst = ct_poly(c, inner, p) + (size_t)li * N;
                    for (size_t k = 0; k < N; k++) dst[k] = addmod(dst[k], mulmod(pt[k], src[k], q), q);
                }
            }
        }
        if (fail || !inner) continue;
        if (i != 0) {
            /* giant rotation in the hoisted form (automorphism applied to the
             * ModUp digits of the inner sum), kept before its ModDown */
            int kk = (int)(((int64_t)g * i * G->s) % n);
            int ga = orc_galois_rot(c, kk), ri = find_rot(c, ga);
            if (ri < 0) { set_err("missing galois key"); orc_ct_free(inner); fail = 1; break; }
            automorph_idx(c, ga, perm);
            uint64_t *X = modup(c, l, ct_poly(c, inner, 1));
            uint64_t *ai = ks_inner(c, l, X, perm, &c->rot[ri]);
            free(X);
            for (int b = 0; b < 2; b++)
                for (int e = 0; e < ne; e++) {
                    uint64_t r = c->q[e < nq ? e : c->L + 1 + (e - nq)];
                    uint64_t *dst = A + ((size_t)b * ne + e) * N;
                    const uint64_t *src = ai + ((size_t)b * ne + e) * N;
                    for (size_t t = 0; t < N; t++) dst[t] = addmod(dst[t], src[t], r);
                }
            free(ai);
            const uint64_t *c0 = ct_poly(c, inner, 0);
            for (int li = 0; li < nq; li++)
                for (size_t t = 0; t < N; t++)
                    E[(size_t)li * N + t] = addmod(E[(size_t)li * N + t], c0[(size_t)li * N + perm[t]], c->q[li]);
            nrot++;
            orc_ct_free(inner);
            continue;
        }
        for (int p2 = 0; p2 < 2; p2++) {
            const uint64_t *src = ct_poly(c, inner, p2);
            for (int li = 0; li < nq; li++)
                for (size_t t = 0; t < N; t++) {
                    size_t e = ((size_t)p2 * nq + li) * N + t;
                    E[e] = addmod(E[e], src[(size_t)li * N + t], c->q[li]);
                }
        }
        if (!acc) acc = inner;   /* giant 0 alone: rescaled below */
        else orc_ct_free(inner);
    }
    free(v); free(coef); free(pt); free(perm);
    for (int k = 0; k < g; k++) orc_ct_free(R[k]);
    free(R);
    orc_ct *r = NULL;
    if (!fail && nrot > 0) {
        r = moddown_rescale(c, l, A, E, x->scale * sd / (double)c->q[l]);
    } else if (!fail && acc) {
        r = orc_rescale(c, acc);
    }
    orc_ct_free(acc);
    free(A); free(E);
    return r;
}

/* ModRaise: the residues mod q_0, lifted to the centred range (-q_0/2, q_0/2]
 * and reduced mod every q_i of level L.  The result decrypts to m + q_0 I
 * with a small integer polynomial I.  Declared scale 2 q_0 Kp, so that
 * CoeffToSlot (whose matrices carry no extra constant) yields the
 * coefficients over q_0 Kp after the conjugate split. */
orc_ct *orc_mod_raise(orc_ctx *c, const orc_ct *a) {
    if (!c->bts) { set_err("bootstrapping not configured"); return NULL; }
    int L = c->L;
    size_t N = c->N;
    uint64_t q0 = c->q[0];
    orc_ct *r = ct_new(c, L, 2.0 * (double)q0 * c->bts->Kp);
    uint64_t *t = malloc(sizeof(uint64_t) * N);
    for (int p = 0; p < 2; p++) {
        memcpy(t, ct_poly(c, a, p), sizeof(uint64_t) * N);
        ntt_inv(c, 0, t);
        for (int i = 0; i <= L; i++) {
            uint64_t *dst = ct_poly(c, r, p) + (size_t)i * N;
            for (size_t k = 0; k < N; k++) {
                int64_t u = t[k] <= (q0 - 1) / 2 ? (int64_t)t[k] : (int64_t)t[k] - (int64_t)q0;
                dst[k] = smod(u, c->q[i]);
            }
            ntt_fwd(c, i, dst);
        }
    }
    free(t);
    return r;
}

/* multiply by the monomial X^k (0 <= k < 2N): exact, no level, same scale.
 * X^(N/2) multiplies every slot by i. */
orc_ct *orc_mul_monomial(orc_ctx *c, const orc_ct *a, int k) {
    size_t N = c->N;
    k %= 2 * c->N; if (k < 0) k += 2 * c->N;
    orc_ct *r = ct_new(c, a->level, a->scale);
    uint64_t *t = malloc(sizeof(uint64_t) * N);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i <= a->level; i++) {
            uint64_t q = c->q[i];
            memcpy(t, ct_poly(c, a, p) + (size_t)i * N, sizeof(uint64_t) * N);
            ntt_inv(c, i, t);
            uint64_t *dst = ct_poly(c, r, p) + (size_t)i * N;
            memset(dst, 0, sizeof(uint64_t) * N);
            for (size_t j = 0; j < N; j++) {
                size_t e = (j + (size_t)k) % (2 * N);
                if (e < N) dst[e] = addmod(dst[e], t[j], q);
                else dst[e - N] = submod(dst[e - N], t[j], q);
            }
            ntt_fwd(c, i, dst);
        }
    free(t);
    return r;
}

/* CoeffToSlot on a ModRaised ciphertext (level L): the three groups with
 * the configured plaintext scales (the scale reduction from the ModRaise
 * scale to S_{L-3}, and with it the precision of the diagonal plaintexts,
 * is shared evenly by the three stages) */
orc_ct *orc_coeff_to_slot(orc_ctx *c, const orc_ct *a) {
    if (!c->bts) { set_err("bootstrapping not configured"); return NULL; }
    if (a->level != c->L) { set_err("CoeffToSlot expects a ModRaised ciphertext"); return NULL; }
    orc_ct *x = ct_copy(c, a);
    for (int t = 0; t < 3 && x; t++) {
        orc_ct *y = lt_apply(c, x, &c->bts->cts[t], c->bts->cts_sd[t]);
        orc_ct_free(x);
        x = y;
    }
    return x;
}
/* SlotToCoeff from the EvalMod output level l_after + 3 down to l_after */
orc_ct *orc_slot_to_coeff(orc_ctx *c, const orc_ct *a) {
    if (!c->bts) { set_err("bootstrapping not configured"); return NULL; }
    if (a->level != c->l_after + 3) { set_err("SlotToCoeff expects the EvalMod output level"); return NULL; }
    orc_ct *x = ct_copy(c, a);
    for (int t = 0; t < 3 && x; t++) {
        orc_ct *y = lt_apply(c, x, &c->bts->stc[t], c->bts->stc_sd[t]);
        orc_ct_free(x);
        x = y;
    }
    return x;
}
/* EvalMod: Chebyshev interpolant of the scaled cosine, then r double angles */
orc_ct *orc_eval_mod(orc_ctx *c, const orc_ct *u) {
    if (!c->bts) { set_err("bootstrapping not configured"); return NULL; }
    orc_ct *y = orc_cheb_eval(c, u, c->bts->cf, c->bts->deg, -1.0, 1.0);
    for (int k = 0; k < c->bts->r && y; k++) {
        orc_ct *sq = mult_rs(c, y, y);
        orc_ct_free(y);
        if (!sq) return NULL;
        orc_ct *t2 = orc_mul_int(c, sq, 2);
        orc_ct_free(sq);
        y = orc_add_const(c, t2, -1.0);
        orc_ct_free(t2);
    }
    return y;
}

/*
 * Bootstrapping of a ciphertext at any level whose message is bounded by the
 * integer M (|m| <= M); its residues mod q_0 are used.  The sine is
 * linearised around the integers and bootstrapping adds an error of fixed
 * size relative to q_0, so the message content is first brought to about
 * s_0 / M with s_0 = q_0 2^-5 by an exact integer multiply:
 *   F    = rint(s_0 / (scale(a) M))   (1 <= F < 2^40)
 *   a'   = F a (mod q_0)
 *   y    = CoeffToSlot(ModRaise(a'))
 *   re   = y + conj(y),  im = -i (y - conj(y))     (-i: monomial X^(3N/2))
 *   e_re = EvalMod(re), e_im = EvalMod(im)
 *   z    = SlotToCoeff(e_re + i e_im)              (i: monomial X^(N/2))
 *   out  = M z (integer multiply), scale(out) = scale(z) ((scale(a) F) M) / s_0
 * Output at level l_afterBTS (the chain's l_after) with the message
 * unchanged; its scale is within about 1/F of S_{l_after}.
 */
orc_ct *orc_bootstrap(orc_ctx *c, const orc_ct *a, int64_t M) {
    if (!c->bts) { set_err("bootstrapping not configured"); return NULL; }
    if (M < 1) { set_err("message bound must be >= 1"); return NULL; }
    int N = c->N;
    double s0 = bts_content_scale(c);
    double Fd = rint(s0 / (a->scale * (double)M));
    if (!(Fd >= 1.0 && Fd < 1099511627776.0)) { set_err("input scale out of range for bootstrapping"); return NULL; }
    orc_ct *a0 = orc_drop_level(c, a, 0);
    if (!a0) return NULL;
    orc_ct *aF = mul_int64(c, a0, (int64_t)Fd, a0->scale);
    orc_ct_free(a0);
    orc_ct *raised = orc_mod_raise(c, aF);
    orc_ct_free(aF);
    orc_ct *y = raised ? orc_coeff_to_slot(c, raised) : NULL;
    orc_ct_free(raised);
    if (!y) return NULL;
    orc_ct *yc = orc_conjugate(c, y);
    if (!yc) { orc_ct_free(y); return NULL; }
    orc_ct *sum = orc_add(c, y, yc), *dif = orc_sub(c, y, yc);
    orc_ct_free(y); orc_ct_free(yc);
    orc_ct *im = orc_mul_monomial(c, dif, 3 * N / 2);
    orc_ct_free(dif);
    orc_ct *er = orc_eval_mod(c, sum);
    orc_ct *ei = er ? orc_eval_mod(c, im) : NULL;
    orc_ct_free(sum); orc_ct_free(im);
    if (!er || !ei) { orc_ct_free(er); orc_ct_free(ei); return NULL; }
    orc_ct *eii = orc_mul_monomial(c, ei, N / 2);
    orc_ct_free(ei);
    orc_ct *w = orc_add(c, er, eii);
    orc_ct_free(er); orc_ct_free(eii);
    if (!w) return NULL;
    orc_ct *z = orc_slot_to_coeff(c, w);
    orc_ct_free(w);
    if (!z) return NULL;
    orc_ct *out = mul_int64(c, z, M, z->scale * (((a->scale * Fd) * (double)M) / s0));
    orc_ct_free(z);
    return out;
}

/*
 * CryptoInvSqrt (paper Alg. 1) for x in [a, b] subset (0, 1]:
 *   ct_x = Mul_P(x, 0.5)                       (lands on S_{l-1})
 *   y    = ChebyshevApprox(x, d) on [a, b]
 *   if literal: y = BTS(y)
 *   repeat n times: [lazy policy: y = BTS(y) when l_y < 2]
 *                   y = NewtonStep(y, ct_x)
 * Pre-BTS (the paper's c = 1): when asked for (pre_bts), or when x has fewer
 * than cheb_depth(d) + 1 levels (the affine map and the Chebyshev tree) or
 * fewer than 3 (ct_x needs 2 for Newton), x is bootstrapped first, with
 * message bound 16 ceil(b).
 * x itself is never bootstrapped otherwise (the c = 0 path).  y is
 * bootstrapped with message bound bts_bound (0: 16 ceil(1 / sqrt(a)), y ~
 * 1/sqrt(x) <= 1/sqrt(a)); the factor 16 keeps the message well inside the
 * range where the sine is linear (the constant coefficient, the slot mean,
 * is the largest).
 * The last Newton step takes x/2 directly from the (possibly bootstrapped)
 * input ciphertext: its limbs are dropped to the step's level and the
 * halving is the exact scale change scale(x) -> 2 scale(x), with no rescale,
 * so x keeps the precision of its own scale.
 * Pre-normalisation by B > 0 (§2.3; B = 0 means 1): the method runs on
 * u = x/B over [a/B, b/B] and the result is scaled back by k = 1/sqrt(B)
 * (the paper's "scale back by sqrt(B)" read as the division the mathematics
 * needs):
 *   - the Chebyshev coefficients interpolate 1/sqrt on [a/B, b/B]; the
 *     affine map is formed from [a, b] on x, which is the same map on u,
 *     so the division by B costs no Mul_P of its own;
 *   - ct_x = Mul_P(x, 0.5/B);
 *   - the last Newton step takes u/2 from the input as the scale change
 *     scale(x) -> 2 B sqrt(B) scale(x) (x operand k u / 2) with the constant
 *     1.5 k, so it yields k y';  with no Newton step the coefficients are
 *     multiplied by k instead.
 *   - the message bound of y's bootstrap is 16 ceil(1/sqrt(a/B)).
 */
orc_ct *orc_invsqrt(orc_ctx *c, const orc_ct *x, int d, int iters, double a, double b, int literal,
                    int64_t bts_bound, int pre_bts, double B) {
    if (!(B >= 0) || !isfinite(B)) { set_err("bad pre-normalisation constant"); return NULL; }
    const double Bn = B > 0 ? B : 1.0, an = a / Bn, bn = b / Bn, kappa = 1.0 / sqrt(Bn);
    double *cf = malloc(sizeof(double) * (d + 1));
    if (d < 1 || iters < 0 || !(a > 0) || !(b > a) || orc_cheb_coeffs_invsqrt(d, an, bn, cf) != 0) {
        free(cf); set_err("bad degree / iterations / interval"); return NULL;
    }
    if (iters == 0)
        for (int k = 0; k <= d; k++) cf[k] *= kappa;
    orc_ct *xb = NULL;
    const int64_t My = bts_bound > 0 ? bts_bound : 16 * (int64_t)ceil(1.0 / sqrt(an));
    /* the ciphertext the chain reads holds x / s: s = 1, or s = B once x has
       been pre-normalised by a homomorphic product with 1/B ahead of a
       Pre-BTS, so that the bootstrap sees a message bounded by b/B */
    double s = 1.0;
    if (pre_bts || x->level < cheb_depth(d) + 1 || x->level < 3) {
        if (!c->bts) {
            if (pre_bts || x->level < 2) { free(cf); set_err("level"); return NULL; }
        } else {
            orc_ct *xn = NULL;
            if (Bn > 1.0) {
                xn = orc_mul_const_down(c, x, 1.0 / Bn);
                if (!xn) { free(cf); return NULL; }
                x = xn;
                s = Bn;
            }
            xb = orc_bootstrap(c, x, 16 * (int64_t)ceil(b / s));
            orc_ct_free(xn);
            if (!xb) { free(cf); return NULL; }
            x = xb;
        }
    }
    orc_ct *cx = mul_const_down(c, x, 0.5 * s / Bn);
    orc_ct *y = orc_cheb_eval(c, x, cf, d, a / s, b / s);
    free(cf);
    if (!cx || !y) { orc_ct_free(cx); orc_ct_free(y); orc_ct_free(xb); return NULL; }
    if (literal) {
        orc_ct *t = orc_bootstrap(c, y, My);
        orc_ct_free(y);
        if (!t) { orc_ct_free(cx); orc_ct_free(xb); return NULL; }
        y = t;
    }
    for (int i = 0; i < iters; i++) {
        if (y->level < 2) {
            if (cx->level < 2) { orc_ct_free(y); orc_ct_free(cx); orc_ct_free(xb); set_err("level"); return NULL; }
            orc_ct *t = orc_bootstrap(c, y, My);
            orc_ct_free(y);
            if (!t) { orc_ct_free(cx); orc_ct_free(xb); return NULL; }
            y = t;
        }
        orc_ct *yn;
        if (i == iters - 1) {
            orc_ct *xr = ct_copy(c, x);
            xr->scale = x->scale * (2.0 * (Bn / s) * sqrt(Bn));
            yn = newton_step(c, y, xr, 1, 1.5 * kappa);
            orc_ct_free(xr);
        } else {
            yn = orc_newton_step(c, y, cx);
        }
        orc_ct_free(y);
        if (!yn) { orc_ct_free(cx); orc_ct_free(xb); return NULL; }
        y = yn;
    }
    orc_ct_free(cx);
    orc_ct_free(xb);
    return y;
}
