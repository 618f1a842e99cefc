// gpu.h -- launch interface of the HIP kernels (kernels.hip) used by the host
// orchestration (ckks_lib.hip).  Device data layout: every polynomial is a
// sequence of limbs of N uint64 words; a "batch" of limbs is contiguous with
// limb stride N.  Each launch names, for each limb of a poly, the index of its
// prime in the chain q_0..q_L, p_0..p_{K-1} (LimbMap); a batch may hold
// several polys with the same limb -> prime map (npoly copies).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gpu {

constexpr int kMaxLimbs = 96;

struct DevPrime {
    uint64_t q;
    uint64_t mu;        // floor(2^(2n) / q), n = bit length of q
    uint64_t mu2_lo;    // floor(2^128 / q), low word
    uint64_t mu2_hi;    //                  high word
    uint32_t nbits;
    uint32_t pad;
};

struct LimbMap {
    uint8_t p[kMaxLimbs];
};

// per-prime twiddle tables, all [np][N]:
//   fw[i][k] = psi_i^br(k),  iw[i][k] = psi_i^-br(k), with Shoup quotients
struct Tables {
    const DevPrime *primes;   // [np]
    const uint64_t *fw, *fw_sh, *iw, *iw_sh;
    const uint64_t *ninv, *ninv_sh;   // [np]
    // binary64 forms for the N = 2^16 transforms of primes below 2^fp_bits:
    // twiddles w and w / q ([np][N]), per prime {q, 1/q, N^-1, N^-1 / q}
    const double *fw_d, *fwq_d, *iw_d, *iwq_d;
    const double *pd;         // [np][4]
    int fp_bits;              // 0: every prime on the integer path
    int logN;
    // N = 2^16 transforms: calls of at most ntt_r4_max (ntt_r8_max) limbs in
    // total use 4 (8) words per thread, larger ones 16; 4-word calls of at
    // most ntt_s4_max limbs put 4 sub-transforms in a block instead of 16
    int ntt_r4_max, ntt_r8_max, ntt_s4_max;
};

// Forward N = 2^16 NTT with a fused source and epilogue (rescale / ModRaise):
//   lift (non-null): the input of limb e of poly p is the centred lift of
//     t[p * t_stride + j] (coefficient form mod q_top) to limb e's prime,
//     instead of work's contents;
//   epi (non-null): the transform's output x is not stored in work; instead
//     out[p][e][j] = (c[p * c_stride + e * N + j] - x) * inv[e] mod q_e
//     (inv / inv_sh: per-limb constant and Shoup quotient, device arrays),
//     plus add[p][e][j] (same layout as out) when add is non-null and bit
//     (p & 1) of add_mask is set (ModDown's finish).
// work ([npoly][nlimb][N]) holds the intermediate between the two passes.
struct NttLift {
    const uint64_t *t;
    size_t t_stride;
    int top;
};
struct NttEpi {
    uint64_t *out;
    const uint64_t *c;
    size_t c_stride;
    const uint64_t *inv, *inv_sh;
    const uint64_t *add;
    int add_mask;
    // optional: add read with a per-poly stride of add_stride words (0: out's
    // layout) and multiplied by add_w[e] (Shoup quotient add_wsh[e]) first
    size_t add_stride;
    const uint64_t *add_w, *add_wsh;
};
void ntt16_fwd_fused(const Tables &T, uint64_t *work, const NttLift *lift, const NttEpi *epi, int nlimb, int npoly,
                     const LimbMap &m, hipStream_t s);

// Batched in-place NTT / inverse NTT of nlimb * npoly limbs.
void ntt(const Tables &T, uint64_t *data, int nlimb, int npoly, const LimbMap &m, bool inverse,
         hipStream_t s);
// Out-of-place form: dst = NTT(src) (src may equal dst).  Source poly p,
// limb e is at src + p * src_poly_stride + e * N (0 = contiguous); dst is
// contiguous.
void ntt_oop(const Tables &T, uint64_t *dst, const uint64_t *src, size_t src_poly_stride, int nlimb, int npoly,
             const LimbMap &m, bool inverse, hipStream_t s);

// Elementwise (all over nlimb limbs x npoly polys with limb map m):
// out = a + b / a - b
void add(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *b, int nlimb, int npoly,
         const LimbMap &m, bool sub, hipStream_t s);
// out[l] = a[l] * c[l] mod q (per-limb constant with Shoup quotient)
struct LimbConsts {
    uint64_t v[kMaxLimbs];
    uint64_t sh[kMaxLimbs];
};
struct LimbWords {
    uint64_t v[kMaxLimbs];
};
void mul_scalar(const Tables &T, uint64_t *out, const uint64_t *a, const LimbConsts &c, int nlimb,
                int npoly, const LimbMap &m, hipStream_t s);
// out[l] = a[l] + c[l] on even-indexed polys (poly 0 of each ciphertext); odd polys copied
void add_scalar(const Tables &T, uint64_t *out, const uint64_t *a, const LimbConsts &c, int nlimb,
                int npoly, const LimbMap &m, hipStream_t s);
// out[l] = k[l] a[l], plus c[l] on even-indexed polys: mul_scalar and add_scalar in one pass
void mul_add_scalar(const Tables &T, uint64_t *out, const uint64_t *a, const LimbConsts &k, const LimbWords &c,
                    int nlimb, int npoly, const LimbMap &m, hipStream_t s);
// out[l][j] = a[l][perm[j]]
void permute(const Tables &T, uint64_t *out, const uint64_t *a, const int32_t *perm, int nlimb, int npoly,
             hipStream_t s);
// tensor of nct ciphertext pairs a, b ([nct][2][nlimb][N]):
// d01 = (a0 b0, a0 b1 + a1 b0) laid out [nct][2][nlimb][N], d2 = a1 b1 [nct][nlimb][N]
void tensor(const Tables &T, uint64_t *d01, uint64_t *d2, const uint64_t *a, const uint64_t *b, int nlimb, int nct,
            const LimbMap &m, hipStream_t s);
// the same tensor with the operands gathered from several ciphertext objects:
// ciphertext k of the product reads a[k / per_src] (and b[...]) at member
// k % per_src (each source holds per_src ciphertexts [per_src][2][nlimb][N])
constexpr int kMaxGather = 16;
struct GatherPtrs {
    const uint64_t *a[kMaxGather];
    const uint64_t *b[kMaxGather];
    int per_src;
};
void tensor_gather(const Tables &T, uint64_t *d01, uint64_t *d2, const GatherPtrs &g, int nlimb, int nct,
                   const LimbMap &m, hipStream_t s);
// dst_p += k * src_p (mod q_prime) over one limb of npoly polys (poly p at
// dst + p * dst_stride, src + p * src_stride)
void add_scaled_limb(const Tables &T, uint64_t *dst, size_t dst_stride, const uint64_t *src, size_t src_stride,
                     int npoly, int prime, uint64_t k, uint64_t k_sh, hipStream_t s);
// out_p,e = (c_p,e - z_p,e) inv[e] + a_p,e w[e]  (mod q_e) over nlimb limbs of
// npoly polys: c at stride c_stride per poly, a at a_stride, z and out
// contiguous [npoly][nlimb][N]; inv / w with Shoup quotients, device arrays
void sub_mul_add_scaled(const Tables &T, uint64_t *out, const uint64_t *c, size_t c_stride, const uint64_t *z,
                        const uint64_t *a, size_t a_stride, const uint64_t *inv, const uint64_t *inv_sh,
                        const uint64_t *w, const uint64_t *w_sh, int nlimb, int npoly, const LimbMap &m,
                        hipStream_t s);
// out = a * b (pointwise), nlimb x npoly
void mul_pointwise(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *b, int nlimb,
                   int npoly, const LimbMap &m, hipStream_t s);
// out = a * b + c (pointwise), nlimb limbs
void mul_add(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *b, const uint64_t *c,
             int nlimb, const LimbMap &m, hipStream_t s);
// out = c - a * b (pointwise) [+ extra * k_l for limbs flagged in `flag`]
void key_combine(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *s_, const uint64_t *e,
                 const uint64_t *sprime, const LimbConsts &k, const uint8_t *flag_host, int nlimb,
                 const LimbMap &m, hipStream_t s);
// signed 64-bit coefficients -> residues for every limb
void signed_to_residues(const Tables &T, uint64_t *out, const int64_t *src, int nlimb, const LimbMap &m,
                        hipStream_t s);

// Rescale helpers.  lift: from t (coef domain, mod q_top) build u_i for
// limbs 0..nlimb-1 (2 polys: t0,t1 -> u[2][nlimb]) as the centred lift.
void rescale_lift(const Tables &T, uint64_t *u, const uint64_t *t, int top_prime, int nlimb, int npoly,
                  size_t t_poly_stride, hipStream_t s);
// out_i = (c_i - u_i) * inv_i  (inv per limb with Shoup)
void sub_mul(const Tables &T, uint64_t *out, const uint64_t *c, const uint64_t *u, const LimbConsts &inv,
             int nlimb, int npoly, size_t c_poly_stride, const LimbMap &m, hipStream_t s);

// Fast base conversion.  in: din limbs (coef domain, primes pin[]),
// out: dout limbs (primes pout[]), out_r = sum_i [in_i * hinv_i]_{q_i} * mat[i][r] mod p_r.
// npoly polys (in stride din*N, out stride dout*N).  mat is device [din][dout].
struct BconvArgs {
    LimbMap pin, pout;
    int din, dout;
    const uint64_t *hinv, *hinv_sh;   // device [din]
    const uint64_t *mat;              // device [dout][din]: output-major, one output's row contiguous
    int split;                        // every input and output prime below 2^60 (30-bit split products)
};
void bconv(const Tables &T, uint64_t *out, const uint64_t *in, const BconvArgs &a, int npoly,
           size_t in_poly_stride, size_t out_poly_stride, hipStream_t s);

// Key inner product over nct ciphertexts: acc[ct][p][e] = sum_j x_j[ct][e] * key_j[p][prime(e)]
// (with perm: x_j read at word perm[j] of each limb, keys at word j)
// (p = 0, 1; acc laid out [nct][2][ne][N]), where
// x_j[ct][e] = e in [lo_j, hi_j) ? dsrc[ct][e] : ext_j[ct][compact(e)],
// compact(e) = e < lo_j ? e : e - (hi_j - lo_j).  Each key word is loaded once
// per thread and used for every ciphertext of the batch.
constexpr int kMaxDigits = 32;
struct InnerArgs {
    int ndig, nct;
    int lo[kMaxDigits], hi[kMaxDigits];
    const uint64_t *ext[kMaxDigits];
    size_t ext_stride[kMaxDigits];
    const uint64_t *dsrc;
    size_t dsrc_stride;
    const uint64_t *key;   // [dnum][2][np][N]
    int np;
    LimbMap m;             // extended basis map (Q_l then P)
    int ne;
    const int32_t *perm;   // nullable: digits read at perm[j] (automorphism of hoisted digits)
};
void key_inner(const Tables &T, uint64_t *acc, const InnerArgs &a, hipStream_t s);

// ModDown finish over nct ciphertexts (2 polys each, poly index p = 2 ct + b):
// out_p,i = (acc_p,i - z_p,i) * Pinv_i, plus add_p,i when bit (p & 1) of add_mask is set.
void moddown_finish(const Tables &T, uint64_t *out, const uint64_t *acc, size_t acc_poly_stride,
                    const uint64_t *z, const uint64_t *add, int add_mask, const LimbConsts &pinv, int nlimb, int nct,
                    const LimbMap &m, hipStream_t s);

// Plaintext-ciphertext multiply-accumulate: out[p][l] = sum_t pt_t[l] * x_t[p][l]
// over npoly polys of nlimb limbs (x_t poly stride nlimb N, same layout as
// out); each plaintext pt_t ([nlimb][N]) is shared by all polys.  The
// products are summed in 128 bits and reduced once (primes < 2^61, nterm
// <= kMaxMac).
constexpr int kMaxMac = 16;
struct MacArgs {
    int nterm;
    const uint64_t *pt[kMaxMac];
    const uint64_t *x[kMaxMac];
};
void pt_mac(const Tables &T, uint64_t *out, const MacArgs &a, int nlimb, int npoly, const LimbMap &m,
            hipStream_t s);

// All giant-step inner sums of a baby-step giant-step transform in one pass:
// out[k][member][p] = sum_b pt[k][b] * x_b[member][p] over the babies b with a
// plaintext (pt[k][b] non-null), p = 0, 1; every baby word is read once.
// Layouts: x_b and out[k] as ciphertext batches [B][2][nlimb][N] (out[k] at
// out + k * gstride); plaintexts [nlimb][N].
constexpr int kMaxBaby = 16, kMaxGiant = 16;
struct GiantArgs {
    int nb, ng;
    const uint64_t *x[kMaxBaby];
    const uint64_t *pt[kMaxGiant][kMaxBaby];
};
void pt_mac_giants(const Tables &T, uint64_t *out, size_t gstride, const GiantArgs &a, int nlimb, int B,
                   const LimbMap &m, hipStream_t s);

// Rotation key-switch jobs over one ModUp of nct inputs: job t applies key
// key[t] to the B inputs ct0[t] .. ct0[t]+B-1, reading their digits through
// perm[t] (the automorphism's NTT-domain index map).  acc is laid out
// [njob][B][2][ne][N].  Each key word is loaded once per job and used for the
// job's B inputs.
constexpr int kMaxJobs = 32;
// terms a summing inner product (key_inner_jobs_sum) may add in 128 bits
// before reducing, at most: the host allows T terms per launch with
// T (q_max - 1)^2 < 2^127 (128 for primes below 2^60, 32 below 2^61) and
// splits longer job lists into launches of at most T / ndig jobs
constexpr int kMaxSumTerms = 128;
struct KsJobs {
    int njob, B;
    int ct0[kMaxJobs];
    const uint64_t *key[kMaxJobs];
    const int32_t *perm[kMaxJobs];
};
void key_inner_jobs(const Tables &T, uint64_t *acc, const InnerArgs &a, const KsJobs &j, hipStream_t s);
// the jobs' inner products summed into one accumulator [B][2][ne][N]
// (added to its contents when accumulate is set)
void key_inner_jobs_sum(const Tables &T, uint64_t *acc, const InnerArgs &a, const KsJobs &j, bool accumulate,
                        hipStream_t s);
// ModDown finish of rotation jobs: out[t] ([B][2][nlimb][N]) receives
// (acc - z) * Pinv for job t, plus on poly 0 the word add[t][...][perm[t][j]]
// (the rotated c0 of the job's input, [B][2][nlimb][N]) when add[t] is set.
struct FinishJobs {
    uint64_t *out[kMaxJobs];
    const uint64_t *add[kMaxJobs];
    const int32_t *perm[kMaxJobs];
};
void moddown_finish_jobs(const Tables &T, const FinishJobs &f, const uint64_t *acc, size_t acc_poly_stride,
                         const uint64_t *z, const LimbConsts &pinv, int nlimb, int njob, int B, const LimbMap &m,
                         hipStream_t s);
// the jobs' rotated c0 summed: out ([B][2][nlimb][N]) = base + on poly 0
// sum_t add[t][...][perm[t][j]], base = out itself (accumulate), extra or zero
void rot_c0_sum(const Tables &T, const FinishJobs &f, uint64_t *out, const uint64_t *extra, bool accumulate,
                int nlimb, int njob, int B, const LimbMap &m, hipStream_t s);

// Linear combination of ciphertext objects at (possibly) different levels:
// out[b][p][l] = sum_t k_t * x_t[b][p][l] over the nlimb lowest limbs (signed
// integer constants k_t, reduced per prime in the kernel; products summed in
// 128 bits, reduced once; nterm <= kMaxComb).  x_t has member stride
// member_stride[t] and poly stride poly_stride[t] (words).
constexpr int kMaxComb = 16;
struct CombArgs {
    int nterm;
    const uint64_t *x[kMaxComb];
    size_t member_stride[kMaxComb];
    size_t poly_stride[kMaxComb];
    int64_t k[kMaxComb];
};
void lincomb(const Tables &T, uint64_t *out, const CombArgs &a, int nlimb, int B, const LimbMap &m, hipStream_t s);
// Several linear combinations of the same terms at once (the baby-step sums of
// one Chebyshev evaluation): out[s] = sum_t k[s][t] * x_t, each term read once
// for every sum; out[s] starts at out + s * out_stride.  Needs N >= 512 (the
// host falls back to one lincomb per sum otherwise); nsum <= kMaxSum.
constexpr int kMaxSum = 8;
struct CombMultiArgs {
    CombArgs c;               // terms (c.k unused)
    int nsum;
    size_t out_stride;
    int64_t k[kMaxSum][kMaxComb];
};
void lincomb_multi(const Tables &T, uint64_t *out, const CombMultiArgs &a, int nlimb, int B, const LimbMap &m,
                   hipStream_t s);

// decryption: m = c0 + c1 * s
void decrypt_combine(const Tables &T, uint64_t *m, const uint64_t *c0, const uint64_t *c1, const uint64_t *sk,
                     int nlimb, const LimbMap &m_, hipStream_t s);
// butterfly-rate probe: `threads` (a multiple of 256) threads, `rounds` rounds
// of 12 forward butterflies each; form 0 = 64-bit words, 1 = binary64, 2 = 32-bit
void butterfly_rate(int form, uint64_t *io, size_t threads, int rounds, uint64_t q, uint64_t w, uint64_t wsh,
                    uint64_t inv64, double wd, double wq, double qinv, hipStream_t s);

}  // namespace gpu
