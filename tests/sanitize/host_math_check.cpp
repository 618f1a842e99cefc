// Exercises the library's host-side set-up arithmetic (host_math.cpp: prime
// chains, roots, SHAKE-256 and the samplers, the canonical embedding, the
// slot-transform plans, the Chebyshev interpolants), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2606_10477_amd/csrc/host_math.h"

int main() {
    // prime chains of the named sets (and a small bootstrapping one)
    struct S { int logN, L, K; hm::ChainShape sh; };
    std::vector<S> sets = {{12, 13, 1, {13, 0, 0, 0, 0}}, {16, 27, 7, {27, 0, 0, 0, 0}},
                           {16, 23, 7, {8, 3, 9, 3, 52}}, {8, 20, 2, {5, 3, 9, 3, 52}}};
    for (const S &s : sets) {
        std::vector<uint64_t> q;
        std::vector<double> ladder;
        hm::prime_chain(s.logN, s.L, s.K, 40, 60, 60, s.sh, q, ladder);
        for (uint64_t p : q) {
            if (!hm::is_prime(p)) return 2;
            const uint64_t r = hm::root_2n(p, 1 << s.logN);
            if (hm::powmod(r, (uint64_t)1 << s.logN, p) != p - 1) return 3;
            if (hm::mulmod(hm::invmod(r, p), r, p) != 1) return 4;
        }
    }
    // SHAKE-256 and the samplers
    std::vector<uint8_t> msg(300), out(700);
    for (int i = 0; i < 300; ++i) msg[i] = (uint8_t)(i * 13);
    hm::shake256(msg.data(), msg.size(), out.data(), out.size());
    const int N = 1 << 10;
    hm::Shake256 x(12345, hm::stream_tag(hm::kKeyA, 5, 1));
    std::vector<uint64_t> u(N);
    hm::uniform_residues(x, 1152921504606584833ull, N, u.data());
    std::vector<int8_t> t(N);
    hm::ternary(x, N, t.data());
    hm::hamming_ternary(x, N, 64, t.data());
    hm::Cdt cdt = hm::gaussian_table(3.2);
    std::vector<int64_t> e(N);
    hm::gaussian(x, cdt, N, e.data());
    // canonical embedding round trip against one prime
    const int logN = 10, n = N / 2;
    std::vector<double> re(n), im(n), re2(n), im2(n);
    for (int i = 0; i < n; ++i) re[i] = std::sin(0.01 * i), im[i] = std::cos(0.02 * i);
    std::vector<int64_t> coef(N);
    if (!hm::encode(logN, re.data(), im.data(), n, std::ldexp(1.0, 40), coef.data())) return 5;
    std::vector<uint64_t> q;
    std::vector<double> ladder;
    hm::prime_chain(logN, 2, 1, 40, 60, 60, hm::ChainShape{2, 0, 0, 0, 0}, q, ladder);
    std::vector<uint64_t> res(2 * (size_t)N);
    for (int l = 0; l < 2; ++l)
        for (int i = 0; i < N; ++i) {
            const int64_t v = coef[i];
            res[(size_t)l * N + i] = v >= 0 ? (uint64_t)v % q[l] : q[l] - ((uint64_t)(-v) % q[l]);
        }
    hm::decode_residues(logN, res.data(), 2, q.data(), std::ldexp(1.0, 40), re2.data(), im2.data());
    double err = 0;
    for (int i = 0; i < n; ++i) err = std::fmax(err, std::fabs(re2[i] - re[i]) + std::fabs(im2[i] - im[i]));
    if (err > 1e-9) return 6;
    // slot-transform plans (three groups of each direction at N = 2^10)
    const int logn = logN - 1;
    int top = logn;
    for (int g = 0; g < 3; ++g) {
        const int sz = logn / 3 + (g < logn % 3 ? 1 : 0);
        int ks[32], kr[32];
        for (int i = 0; i < sz; ++i) ks[i] = top - i, kr[i] = top - sz + 1 + i;
        hm::LtGroupPlan a, b;
        if (!hm::lt_group(logN, ks, sz, true, q[0], 0.0, std::ldexp(1.0, 40), a)) return 7;
        if (!hm::lt_group(logN, kr, sz, false, q[0], g == 2 ? std::ldexp((double)q[0], -5) : 0.0,
                          std::ldexp(1.0, 40), b))
            return 8;
        top -= sz;
    }
    // Chebyshev interpolants
    std::vector<double> cf(128);
    hm::cheb_invsqrt(127, std::ldexp(1.0, -10), 1.0, cf.data());
    hm::cheb_cosmod(31, 25.0, 16.0, cf.data());
    std::printf("host math: chains, samplers, embedding (round-trip error %.2g), plans, interpolants ok\n", err);
    return 0;
}
