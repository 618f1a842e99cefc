// host_math.cpp -- host-side set-up arithmetic of the GPU library.
//
// Built with g++ (it needs libquadmath, which the HIP host compiler lacks) and
// linked into libckks_hip.so.  Everything here runs once per context, key or
// encoded constant; nothing runs per homomorphic operation.
//
// Conventions (each reproduced independently by the CPU oracle):
//  * prime chain: q_0 = largest prime < 2^q0_bits with q = 1 (mod 2N); q_L..q_1
//    top-down, each the unused prime = 1 (mod 2N) nearest to S_l^2 / 2^log_scale
//    (nearest below vs nearest above; ties to the lower), S_L = 2^log_scale,
//    S_{l-1} = (S_l * S_l) / q_l in binary64; special primes descending below q_0.
//  * psi = g^((q-1)/2N) for the least g >= 2 with psi^N = -1.
//  * randomness: SHAKE-256 over (seed as 8 LE bytes || tag as 8 LE bytes).
//  * encoding: slot j <-> zeta^(5^j mod 2N), zeta = exp(i pi / N); the integer
//    coefficients are rint(scale * exact inverse embedding), evaluated in
//    __float128 so that the rounding matches the exact value.
#include "host_math.h"

#include <cmath>
#include <cstring>
#include <quadmath.h>
#include <algorithm>
#include <map>
#include <thread>

namespace hm {

typedef unsigned __int128 u128;
typedef __float128 quad;

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t acc = 1 % q, base = a % q;
    for (; e; e >>= 1) {
        if (e & 1) acc = mulmod(acc, base, q);
        base = mulmod(base, base, q);
    }
    return acc;
}
uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }

// Miller-Rabin; the witnesses 2..37 decide every 64-bit integer.
static bool mr_witness(uint64_t n, uint64_t a, uint64_t d, int r) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) return false;
    while (--r > 0) {
        x = mulmod(x, x, n);
        if (x == n - 1) return false;
    }
    return true;   // a proves n composite
}
bool is_prime(uint64_t n) {
    const uint64_t W[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t w : W) {
        if (n == w) return true;
        if (n % w == 0) return false;
    }
    uint64_t d = n - 1;
    int r = 0;
    while (!(d & 1)) { d >>= 1; ++r; }
    for (uint64_t w : W)
        if (mr_witness(n, w, d, r)) return false;
    return true;
}

// unused prime = 1 (mod step) nearest to T (first below vs first above; ties
// to the lower)
static uint64_t nearest_prime(double T, uint64_t step, const std::vector<uint64_t> &taken_list) {
    auto taken = [&](uint64_t c) { return std::find(taken_list.begin(), taken_list.end(), c) != taken_list.end(); };
    uint64_t t = (uint64_t)std::floor(T);
    uint64_t below = ((t - 1) / step) * step + 1;     // <= t, = 1 mod step
    uint64_t above = below + step;
    while (!is_prime(below) || taken(below)) below -= step;
    while (!is_prime(above) || taken(above)) above += step;
    return ((double)above - T < T - (double)below) ? above : below;
}

// Computation levels A..1 (A = l_after) top-down from S_A = 2^log_scale with
// q_l nearest to S_l^2 / 2^log_scale.  A bootstrapping chain then adds the
// EvalMod levels (same rule from S_E = 2^bts_bits at E = A + n_stc + n_evm,
// down to level A + n_stc), the SlotToCoeff primes (levels A+1..A+n_stc,
// nearest to 2^log_scale, S = 2^log_scale below the EvalMod output) and the
// CoeffToSlot primes (levels E+1..L, nearest to 2^bts_bits, S = 2^bts_bits),
// in that order, then the special primes below 2^p_bits.
void prime_chain(int logN, int L, int K, int log_scale, int q0_bits, int p_bits, const ChainShape &shape,
                 std::vector<uint64_t> &primes, std::vector<double> &ladder) {
    const uint64_t step = (uint64_t)2 << logN;   // 2N
    primes.assign(L + 1 + K, 0);
    ladder.assign(L + 1, 0.0);
    std::vector<uint64_t> taken;
    // q_0: walk down from the largest 1 (mod 2N) number below 2^q0_bits
    uint64_t lim = (uint64_t)1 << q0_bits;
    uint64_t c = ((lim - 1) / step) * step + 1;
    if (c >= lim) c -= step;
    while (!is_prime(c)) c -= step;
    primes[0] = c;
    taken.push_back(c);
    auto adaptive = [&](int top, int bot, double D) {
        double S = D;
        ladder[top] = S;
        for (int l = top; l > bot; --l) {
            double T = (S * S) / D;
            uint64_t pick = nearest_prime(T, step, taken);
            primes[l] = pick;
            taken.push_back(pick);
            S = (S * S) / (double)pick;
            ladder[l - 1] = S;
        }
    };
    const double D = std::ldexp(1.0, log_scale);
    const int A = shape.n_evm > 0 ? shape.l_after : L;
    adaptive(A, 0, D);
    if (shape.n_evm > 0) {
        const double Db = std::ldexp(1.0, shape.bts_bits);
        const int E = A + shape.n_stc + shape.n_evm;
        adaptive(E, A + shape.n_stc, Db);
        for (int l = A + 1; l <= A + shape.n_stc; ++l) {
            primes[l] = nearest_prime(D, step, taken);
            taken.push_back(primes[l]);
            if (l < A + shape.n_stc) ladder[l] = D;
        }
        for (int l = E + 1; l <= L; ++l) {
            primes[l] = nearest_prime(Db, step, taken);
            taken.push_back(primes[l]);
            ladder[l] = Db;
        }
    }
    uint64_t plim = (uint64_t)1 << p_bits;
    uint64_t pc = ((plim - 1) / step) * step + 1;
    if (pc >= plim) pc -= step;
    for (int k = 0; k < K; ++k) {
        while (!is_prime(pc) || std::find(taken.begin(), taken.end(), pc) != taken.end()) pc -= step;
        primes[L + 1 + k] = pc;
        taken.push_back(pc);
        pc -= step;
    }
}

uint64_t root_2n(uint64_t q, int N) {
    const uint64_t e = (q - 1) / (2 * (uint64_t)N);
    for (uint64_t g = 2;; ++g) {
        uint64_t r = powmod(g, e, q);
        if (powmod(r, (uint64_t)N, q) == q - 1) return r;
    }
}

// ---------------------------------------------------------------------------
// Keccak-f[1600] / SHAKE-256 (rate 136 bytes, domain suffix 0x1F)
// ---------------------------------------------------------------------------
static const uint64_t kRC[24] = {
    0x0000000000000001ULL, 0x0000000000008082ULL, 0x800000000000808AULL, 0x8000000080008000ULL,
    0x000000000000808BULL, 0x0000000080000001ULL, 0x8000000080008081ULL, 0x8000000000008009ULL,
    0x000000000000008AULL, 0x0000000000000088ULL, 0x0000000080008009ULL, 0x000000008000000AULL,
    0x000000008000808BULL, 0x800000000000008BULL, 0x8000000000008089ULL, 0x8000000000008003ULL,
    0x8000000000008002ULL, 0x8000000000000080ULL, 0x000000000000800AULL, 0x800000008000000AULL,
    0x8000000080008081ULL, 0x8000000000008080ULL, 0x0000000080000001ULL, 0x8000000080008008ULL};
// rotation offset of lane (x, y), indexed x + 5y
static const int kRho[25] = {0, 1, 62, 28, 27, 36, 44, 6, 55, 20, 3, 10, 43,
                             25, 39, 41, 45, 15, 21, 8, 18, 2, 61, 56, 14};
static const size_t kRate = 136;

static inline uint64_t rol(uint64_t v, int r) { return r == 0 ? v : (v << r) | (v >> (64 - r)); }

void Shake256::permute() {
    uint64_t *a = s_;
    for (int round = 0; round < 24; ++round) {
        uint64_t c[5];
        for (int x = 0; x < 5; ++x) c[x] = a[x] ^ a[5 + x] ^ a[10 + x] ^ a[15 + x] ^ a[20 + x];
        for (int x = 0; x < 5; ++x) {
            uint64_t d = c[(x + 4) % 5] ^ rol(c[(x + 1) % 5], 1);
            for (int y = 0; y < 25; y += 5) a[y + x] ^= d;
        }
        uint64_t b[25];
        for (int y = 0; y < 5; ++y)
            for (int x = 0; x < 5; ++x) {
                // pi: lane (x, y) moves to (y, 2x + 3y)
                int nx = y, ny = (2 * x + 3 * y) % 5;
                b[nx + 5 * ny] = rol(a[x + 5 * y], kRho[x + 5 * y]);
            }
        for (int y = 0; y < 5; ++y)
            for (int x = 0; x < 5; ++x)
                a[x + 5 * y] = b[x + 5 * y] ^ (~b[(x + 1) % 5 + 5 * y] & b[(x + 2) % 5 + 5 * y]);
        a[0] ^= kRC[round];
    }
}

static inline void xor_byte(uint64_t *s, size_t pos, uint8_t v) { s[pos >> 3] ^= (uint64_t)v << (8 * (pos & 7)); }
static inline uint8_t get_byte(const uint64_t *s, size_t pos) { return (uint8_t)(s[pos >> 3] >> (8 * (pos & 7))); }

Shake256::Shake256(const uint8_t *msg, size_t len) {
    std::memset(s_, 0, sizeof(s_));
    size_t pos = 0;
    for (size_t i = 0; i < len; ++i) {
        xor_byte(s_, pos, msg[i]);
        if (++pos == kRate) { permute(); pos = 0; }
    }
    xor_byte(s_, pos, 0x1F);
    xor_byte(s_, kRate - 1, 0x80);
    permute();
    off_ = 0;
}
Shake256::Shake256(uint64_t seed, uint64_t tag) : Shake256(nullptr, 0) {
    uint8_t in[16];
    for (int i = 0; i < 8; ++i) { in[i] = (uint8_t)(seed >> (8 * i)); in[8 + i] = (uint8_t)(tag >> (8 * i)); }
    *this = Shake256(in, 16);
}
uint8_t Shake256::byte() {
    if (off_ == kRate) { permute(); off_ = 0; }
    return get_byte(s_, off_++);
}
void Shake256::squeeze(uint8_t *out, size_t len) {
    for (size_t i = 0; i < len; ++i) out[i] = byte();
}
uint32_t Shake256::u32() {
    uint32_t v = 0;
    for (int i = 0; i < 4; ++i) v |= (uint32_t)byte() << (8 * i);
    return v;
}
uint64_t Shake256::u64() {
    uint64_t v = 0;
    for (int i = 0; i < 8; ++i) v |= (uint64_t)byte() << (8 * i);
    return v;
}
void shake256(const uint8_t *msg, size_t len, uint8_t *out, size_t outlen) {
    Shake256 x(msg, len);
    x.squeeze(out, outlen);
}

uint64_t stream_tag(int kind, int galois, int digit) {
    return ((uint64_t)kind << 56) | ((uint64_t)(uint32_t)galois << 16) | (uint64_t)(uint16_t)digit;
}

void uniform_residues(Shake256 &x, uint64_t q, int N, uint64_t *out) {
    const int bits = 64 - __builtin_clzll(q);
    const uint64_t mask = bits == 64 ? ~0ULL : ((1ULL << bits) - 1);
    for (int i = 0; i < N; ++i) {
        uint64_t v = x.u64() & mask;
        while (v >= q) v = x.u64() & mask;
        out[i] = v;
    }
}
void ternary(Shake256 &x, int N, int8_t *out) {
    for (int i = 0; i < N; ++i) {
        uint8_t b = x.byte();
        while (b == 0xFF) b = x.byte();
        out[i] = (int8_t)(b % 3) - 1;
    }
}
void hamming_ternary(Shake256 &x, int N, int h, int8_t *out) {
    std::memset(out, 0, N);
    for (int placed = 0; placed < h;) {
        uint32_t pos = x.u32() & (uint32_t)(N - 1);
        if (out[pos]) continue;
        out[pos] = (x.byte() & 1) ? -1 : 1;
        ++placed;
    }
}
Cdt gaussian_table(double sigma) {
    // thresholds floor(2^53 * P(|e| <= k)), k < J; the last entry is 2^53
    int J = (int)std::ceil(6.25 * sigma);
    if (J > 63) J = 63;
    const double two_var = 2.0 * sigma * sigma;
    std::vector<double> w(J + 1);
    for (int j = 0; j <= J; ++j) w[j] = std::exp(-((double)j * (double)j) / two_var);
    double rest = 0.0;
    for (int j = 1; j <= J; ++j) rest += w[j];
    const double total = w[0] + 2.0 * rest;
    Cdt c;
    c.t.resize(J + 1);
    double cum = 0.0;
    for (int k = 0; k < J; ++k) {
        if (k > 0) cum += w[k];
        c.t[k] = (uint64_t)(((w[0] + 2.0 * cum) / total) * 9007199254740992.0);
    }
    c.t[J] = 1ULL << 53;
    return c;
}
void gaussian(Shake256 &x, const Cdt &cdt, int N, int64_t *out) {
    const int last = (int)cdt.t.size() - 1;
    for (int i = 0; i < N; ++i) {
        uint64_t w = x.u64();
        uint64_t u = w >> 11;
        int k = 0;
        while (k < last && u >= cdt.t[k]) ++k;
        out[i] = (k != 0 && (w & 1)) ? -(int64_t)k : (int64_t)k;
    }
}

// ---------------------------------------------------------------------------
// Canonical embedding (quad precision)
// ---------------------------------------------------------------------------
struct cplx { quad r, i; };
static inline cplx cmul(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

// exp(2 pi i num / den)
static cplx unit_root(long long num, long long den) {
    num %= den;
    if (num < 0) num += den;
    quad th = (2 * M_PIq * (quad)num) / (quad)den;
    return {cosq(th), sinq(th)};
}

// In-place length-n DFT, X_k = sum_t x_t exp(sign 2 pi i t k / n), decimation
// in frequency with a final bit-reversal permutation.
static void dft(std::vector<cplx> &x, int sign) {
    const size_t n = x.size();
    std::vector<cplx> roots(n / 2 + 1);
    for (size_t k = 0; k < n / 2; ++k) roots[k] = unit_root(sign * (long long)k, (long long)n);
    for (size_t half = n / 2; half >= 1; half >>= 1) {
        const size_t stride = n / (2 * half);
        for (size_t start = 0; start < n; start += 2 * half)
            for (size_t j = 0; j < half; ++j) {
                cplx u = x[start + j], v = x[start + j + half];
                x[start + j] = {u.r + v.r, u.i + v.i};
                x[start + j + half] = cmul({u.r - v.r, u.i - v.i}, roots[j * stride]);
            }
        if (half == 1) break;
    }
    int bits = 0;
    while (((size_t)1 << bits) < n) ++bits;
    for (size_t k = 0; k < n; ++k) {
        size_t r = 0, v = k;
        for (int b = 0; b < bits; ++b) { r = (r << 1) | (v & 1); v >>= 1; }
        if (r > k) std::swap(x[k], x[r]);
    }
}

// position of slot j in the length-n DFT: (5^j mod 2N - 1) / 4
static std::vector<size_t> slot_positions(int logN) {
    const uint64_t M = (uint64_t)2 << logN;
    const size_t n = (size_t)1 << (logN - 1);
    std::vector<size_t> pos(n);
    uint64_t g = 1;
    for (size_t j = 0; j < n; ++j) { pos[j] = (size_t)((g - 1) >> 2); g = (g * 5) % M; }
    return pos;
}

static bool encode_slots(int logN, const std::vector<cplx> &z, double scale, int64_t *out) {
    const size_t N = (size_t)1 << logN, n = N / 2;
    const std::vector<size_t> pos = slot_positions(logN);
    std::vector<cplx> G(n);
    for (size_t j = 0; j < n; ++j) G[pos[j]] = z[j];
    dft(G, -1);
    bool ok = true;
    const quad sc = (quad)scale;
    for (size_t k = 0; k < n; ++k) {
        cplx w = cmul(G[k], unit_root(-(long long)k, 2 * (long long)N));
        quad re = rintq(w.r / (quad)n * sc), im = rintq(w.i / (quad)n * sc);
        if (fabsq(re) > 9.2e18Q || fabsq(im) > 9.2e18Q) ok = false;
        out[k] = (int64_t)re;
        out[k + n] = (int64_t)im;
    }
    return ok;
}

bool encode(int logN, const double *re, const double *im, size_t nslots, double scale, int64_t *out) {
    const size_t n = (size_t)1 << (logN - 1);
    std::vector<cplx> z(n, cplx{0, 0});
    for (size_t j = 0; j < nslots && j < n; ++j) z[j] = {(quad)re[j], im ? (quad)im[j] : (quad)0};
    return encode_slots(logN, z, scale, out);
}

// ---------------------------------------------------------------------------
// Bootstrapping slot transforms (quad precision)
// ---------------------------------------------------------------------------
// Butterfly stage k (length len = 2^k, half h) on n slots, as three
// diagonals at offsets 0, +h, -h.  Forward: y_j = x_j + t_j x_{j+h},
// y_{j+h} = x_j - t_j x_{j+h}; inverse: x_j = (y_j + y_{j+h}) / 2,
// x_{j+h} = (y_j - y_{j+h}) / (2 t_j); t_j = exp(2 pi i (5^j mod 4 len) / (4 len)).
static void butterfly_diagonals(size_t n, int k, bool inverse, std::vector<cplx> d[3]) {
    const size_t len = (size_t)1 << k, h = len / 2;
    for (int e = 0; e < 3; ++e) d[e].assign(n, cplx{0, 0});
    std::vector<cplx> tw(h);
    uint64_t p5 = 1;
    for (size_t j = 0; j < h; ++j) {
        tw[j] = unit_root((long long)p5, 4 * (long long)len);
        p5 = (p5 * 5) % (4 * len);
    }
    for (size_t j = 0; j < n; ++j) {
        const size_t jj = j % len;
        if (jj < h) {
            if (!inverse) { d[0][j] = {1, 0}; d[1][j] = tw[jj]; }
            else { d[0][j] = {0.5Q, 0}; d[1][j] = {0.5Q, 0}; }
        } else {
            const cplx t = tw[jj - h];
            if (!inverse) { d[0][j] = {-t.r, -t.i}; d[2][j] = {1, 0}; }
            else { d[2][j] = {t.r / 2, -t.i / 2}; d[0][j] = {-t.r / 2, t.i / 2}; }   // 1/(2t) = conj(t)/2
        }
    }
}

bool lt_group(int logN, const int *ks, int cnt, bool inverse, uint64_t q0, double s0, double sd,
              LtGroupPlan &out) {
    const size_t n = (size_t)1 << (logN - 1);
    // diagonal form of the product, offset (mod n) -> values
    std::map<size_t, std::vector<cplx>> cur;
    cur[0].assign(n, cplx{1, 0});
    int kmin = ks[0], kmax = ks[0];
    std::vector<cplx> d[3];
    for (int t = 0; t < cnt; ++t) {
        const int k = ks[t];
        kmin = std::min(kmin, k);
        kmax = std::max(kmax, k);
        butterfly_diagonals(n, k, inverse, d);
        const size_t h = (size_t)1 << (k - 1);
        const size_t off[3] = {0, h % n, (n - h) % n};
        std::map<size_t, std::vector<cplx>> nxt;
        for (auto &kv : cur)
            for (int e = 0; e < 3; ++e) {
                auto &dst = nxt[(off[e] + kv.first) % n];
                if (dst.empty()) dst.assign(n, cplx{0, 0});
                for (size_t j = 0; j < n; ++j) {
                    cplx v = cmul(d[e][j], kv.second[(j + off[e]) % n]);
                    dst[j].r += v.r;
                    dst[j].i += v.i;
                }
            }
        cur.swap(nxt);
    }
    const quad cm = s0 > 0 ? (quad)q0 / (2 * M_PIq * (quad)s0) : (quad)1;
    const size_t stride = (size_t)1 << (kmin - 1);
    const long long ns = (long long)(n / stride);
    const bool wrap = ns <= (1LL << (kmax - kmin + 1));
    std::vector<std::pair<long long, const std::vector<cplx> *>> diag;
    for (auto &kv : cur) {
        bool nz = false;
        for (const cplx &v : kv.second)
            if (v.r != 0 || v.i != 0) { nz = true; break; }
        if (!nz) continue;
        long long m = (long long)(kv.first / stride);
        if (!wrap && m > ns / 2) m -= ns;
        diag.emplace_back(m, &kv.second);
    }
    std::sort(diag.begin(), diag.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    const long long span = diag.back().first - diag.front().first + 1;
    int e = 0;
    while ((1LL << e) < span) ++e;
    const int g = 1 << ((e + 1) / 2);
    out.stride = (int)stride;
    out.g = g;
    out.terms.assign(diag.size(), LtTerm{});
    std::vector<char> ok(diag.size(), 1);
    auto work = [&](size_t lo, size_t hi) {
        std::vector<cplx> z(n);
        for (size_t t = lo; t < hi; ++t) {
            const long long m = diag[t].first;
            long long gi = m / g;
            if (m % g != 0 && m < 0) --gi;        // floor division
            const long long b = m - gi * g;
            const long long sh = gi * g * (long long)stride;
            const std::vector<cplx> &v = *diag[t].second;
            for (size_t j = 0; j < n; ++j) {
                long long src = (((long long)j - sh) % (long long)n + (long long)n) % (long long)n;
                z[j] = {v[src].r * cm, v[src].i * cm};
            }
            LtTerm &T = out.terms[t];
            T.giant = (int)gi;
            T.baby = (int)b;
            T.coef.resize(2 * n);
            ok[t] = encode_slots(logN, z, sd, T.coef.data());
        }
    };
    const size_t nt = diag.size();
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    const size_t chunk = (nt + hw - 1) / hw;
    for (size_t lo = 0; lo < nt; lo += chunk) th.emplace_back(work, lo, std::min(nt, lo + chunk));
    for (auto &t : th) t.join();
    for (char o : ok)
        if (!o) return false;
    return true;
}

// ---------------------------------------------------------------------------
// Exact CRT (multi-word integer) and decode
// ---------------------------------------------------------------------------
typedef std::vector<uint64_t> big;   // little-endian 64-bit words

static void big_mul_small(const big &a, uint64_t m, big &out) {
    out.assign(a.size() + 1, 0);
    u128 carry = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        u128 t = (u128)a[i] * m + carry;
        out[i] = (uint64_t)t;
        carry = t >> 64;
    }
    out[a.size()] = (uint64_t)carry;
}
static void big_add_to(big &acc, const big &a) {
    if (acc.size() < a.size() + 1) acc.resize(a.size() + 1, 0);
    u128 carry = 0;
    for (size_t i = 0; i < acc.size(); ++i) {
        u128 t = (u128)acc[i] + (i < a.size() ? a[i] : 0) + carry;
        acc[i] = (uint64_t)t;
        carry = t >> 64;
    }
}
static int big_cmp(const big &a, const big &b) {
    size_t n = std::max(a.size(), b.size());
    for (size_t i = n; i-- > 0;) {
        uint64_t x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}
static void big_sub_to(big &acc, const big &a) {   // acc -= a, acc >= a
    u128 borrow = 0;
    for (size_t i = 0; i < acc.size(); ++i) {
        u128 t = (u128)acc[i] - (i < a.size() ? a[i] : 0) - borrow;
        acc[i] = (uint64_t)t;
        borrow = (t >> 64) ? 1 : 0;
    }
}
static quad big_to_quad(const big &a) {
    quad v = 0;
    for (size_t i = a.size(); i-- > 0;) v = v * 18446744073709551616.0Q + (quad)a[i];
    return v;
}

void decode_residues(int logN, const uint64_t *res, int nlimbs, const uint64_t *primes,
                     double scale, double *re, double *im) {
    const size_t N = (size_t)1 << logN, n = N / 2;
    // Q, Qhat_i = Q / q_i and [Qhat_i^-1]_{q_i}
    big Q{1};
    for (int i = 0; i < nlimbs; ++i) { big t; big_mul_small(Q, primes[i], t); Q = t; }
    std::vector<big> Qhat(nlimbs);
    std::vector<uint64_t> Qhat_inv(nlimbs);
    for (int i = 0; i < nlimbs; ++i) {
        big h{1};
        uint64_t hm = 1;
        for (int k = 0; k < nlimbs; ++k) {
            if (k == i) continue;
            big t; big_mul_small(h, primes[k], t); h = t;
            hm = mulmod(hm, primes[k] % primes[i], primes[i]);
        }
        Qhat[i] = h;
        Qhat_inv[i] = invmod(hm, primes[i]);
    }
    big halfQ(Q.size(), 0);   // floor(Q / 2)
    for (size_t i = 0; i < Q.size(); ++i)
        halfQ[i] = (Q[i] >> 1) | (i + 1 < Q.size() ? (Q[i + 1] << 63) : 0);
    std::vector<quad> coef(N);
    big acc, term;
    for (size_t t = 0; t < N; ++t) {
        acc.assign(Q.size() + 2, 0);
        for (int i = 0; i < nlimbs; ++i) {
            uint64_t y = mulmod(res[(size_t)i * N + t], Qhat_inv[i], primes[i]);
            big_mul_small(Qhat[i], y, term);
            big_add_to(acc, term);
        }
        while (big_cmp(acc, Q) >= 0) big_sub_to(acc, Q);
        if (big_cmp(acc, halfQ) > 0) {
            big neg = Q;
            neg.resize(acc.size(), 0);
            big_sub_to(neg, acc);
            coef[t] = -big_to_quad(neg);
        } else {
            coef[t] = big_to_quad(acc);
        }
    }
    // slots: z_j = sum_k (m_k + i m_{k+n}) zeta^(e_j k), e_j = 5^j mod 2N
    std::vector<cplx> F(n);
    for (size_t k = 0; k < n; ++k) F[k] = cmul({coef[k], coef[k + n]}, unit_root((long long)k, 2 * (long long)N));
    dft(F, +1);
    const std::vector<size_t> pos = slot_positions(logN);
    const quad sc = (quad)scale;
    for (size_t j = 0; j < n; ++j) {
        re[j] = (double)(F[pos[j]].r / sc);
        if (im) im[j] = (double)(F[pos[j]].i / sc);
    }
}

// ---------------------------------------------------------------------------
// Chebyshev interpolation at first-kind nodes (quad precision)
// ---------------------------------------------------------------------------
template <class F>
static void cheb_interp(int d, quad a, quad b, F f, double *coeffs) {
    const int n = d + 1;
    std::vector<quad> theta(n), fv(n);
    for (int j = 0; j < n; ++j) {
        theta[j] = M_PIq * ((quad)(2 * j + 1) / (quad)(2 * n));
        fv[j] = f((a + b) / 2 + (b - a) / 2 * cosq(theta[j]));
    }
    for (int k = 0; k <= d; ++k) {
        quad acc = 0;
        for (int j = 0; j < n; ++j) acc += fv[j] * cosq((quad)k * theta[j]);
        acc = 2 * acc / (quad)n;
        coeffs[k] = (double)(k == 0 ? acc / 2 : acc);
    }
}
void cheb_invsqrt(int d, double a, double b, double *coeffs) {
    cheb_interp(d, (quad)a, (quad)b, [](quad x) { return 1 / sqrtq(x); }, coeffs);
}
void cheb_cosmod(int d, double K, double two_r, double *coeffs) {
    const quad Kq = (quad)K, R = (quad)two_r;
    cheb_interp(d, (quad)-1, (quad)1, [&](quad t) { return cosq(2 * M_PIq * (Kq * t - 0.25Q) / R); }, coeffs);
}

}  // namespace hm
