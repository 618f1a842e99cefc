// host_math.h -- host-side set-up arithmetic of the library (compiled by g++,
// see host_math.cpp): prime chain, NTT roots, SHAKE-256 sampling, canonical
// embedding in quad precision, Chebyshev interpolation.  None of this runs on
// the per-ciphertext hot path; it produces tables, keys' random polynomials and
// encoded plaintexts that the HIP kernels then consume.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace hm {

bool is_prime(uint64_t n);
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q);
uint64_t powmod(uint64_t a, uint64_t e, uint64_t q);
uint64_t invmod(uint64_t a, uint64_t q);

// Shape of a bootstrapping chain: levels l_after+1..L are consumed by
// bootstrapping (SlotToCoeff n_stc, EvalMod n_evm, CoeffToSlot n_cts, from
// the bottom up).  n_evm = 0: a plain chain with l_after = L.
struct ChainShape {
    int l_after = 0, n_stc = 0, n_evm = 0, n_cts = 0, bts_bits = 0;
};
// Prime chain q_0..q_L, p_0..p_{K-1} and the canonical scale ladder S_0..S_L.
void prime_chain(int logN, int L, int K, int log_scale, int q0_bits, int p_bits, const ChainShape &shape,
                 std::vector<uint64_t> &primes, std::vector<double> &ladder);
// 2N-th root of unity of q: g^((q-1)/2N) for the least g >= 2 of order 2N.
uint64_t root_2n(uint64_t q, int N);

// SHAKE-256 extendable-output function (FIPS 202).
class Shake256 {
public:
    Shake256(const uint8_t *msg, size_t len);
    Shake256(uint64_t seed, uint64_t tag);
    void squeeze(uint8_t *out, size_t len);
    uint8_t byte();
    uint32_t u32();
    uint64_t u64();
private:
    void permute();
    uint64_t s_[25];
    size_t off_;
};
void shake256(const uint8_t *msg, size_t len, uint8_t *out, size_t outlen);

// Stream tags (kind << 56 | galois << 16 | digit).
enum TagKind { kSecret = 1, kPkA = 2, kPkE = 3, kKeyA = 4, kKeyE = 5, kEncV = 6, kEncE0 = 7, kEncE1 = 8 };
uint64_t stream_tag(int kind, int galois, int digit);

// Samplers (coefficient order 0..N-1).
void uniform_residues(Shake256 &x, uint64_t q, int N, uint64_t *out);
void ternary(Shake256 &x, int N, int8_t *out);
void hamming_ternary(Shake256 &x, int N, int h, int8_t *out);
struct Cdt { std::vector<uint64_t> t; };
Cdt gaussian_table(double sigma);
void gaussian(Shake256 &x, const Cdt &cdt, int N, int64_t *out);

// Canonical embedding.  encode: n = N/2 complex slots (re, im may be shorter:
// zero padded) at `scale` -> N integer coefficients (int64; false if out of range).
bool encode(int logN, const double *re, const double *im, size_t nslots, double scale, int64_t *out);
// decode: residues mod q_0..q_{nlimbs-1} of the plaintext coefficients (row i
// = limb i, N words each, coefficient domain) -> centred integers (exact CRT)
// -> N/2 slots divided by `scale`.
void decode_residues(int logN, const uint64_t *res, int nlimbs, const uint64_t *primes,
                     double scale, double *re, double *im);

// Bootstrapping slot transforms.  One group of butterfly stages (stage k:
// butterflies of length 2^k; ks[] in the order they are applied; inverse
// stages for CoeffToSlot, forward for SlotToCoeff), as a matrix on the N/2
// slots, optionally multiplied by q0 / (2 pi s0) (s0 > 0).  Its nonzero
// diagonals m (offset m * stride slots) are split m = g i + b (0 <= b < g);
// each term's plaintext is diagonal m rotated right by g i stride slots,
// encoded at scale sd.  Returns false if a coefficient does not fit int64.
struct LtTerm {
    int giant, baby;
    std::vector<int64_t> coef;   // N encoded coefficients
};
struct LtGroupPlan {
    int stride = 0, g = 0;
    std::vector<LtTerm> terms;   // ascending m
};
bool lt_group(int logN, const int *ks, int cnt, bool inverse, uint64_t q0, double s0, double sd,
              LtGroupPlan &out);

// Chebyshev interpolant of 1/sqrt on [a, b] (degree d, first-kind nodes).
void cheb_invsqrt(int d, double a, double b, double *coeffs);
// Chebyshev interpolant on [-1, 1] of cos(2 pi (K t - 1/4) / 2^r).
void cheb_cosmod(int d, double K, double two_r, double *coeffs);

}  // namespace hm
