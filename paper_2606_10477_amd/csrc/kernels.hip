// kernels.hip -- gfx950 kernels of the RNS-CKKS hot path.
//
// Arithmetic: every residue is a uint64 word in [0, q), q < 2^62.
//  * constant multiplications (twiddles, per-limb scalars) use Shoup's
//    method with a precomputed quotient w' = floor(w 2^64 / q);
//  * products of two variables use Barrett reduction of the 128-bit product
//    with mu = floor(2^(2n) / q) (n = bit length of q);
//  * sums of products (base conversion, key inner product) accumulate the
//    128-bit products without reduction and reduce once with
//    mu2 = floor(2^128 / q).
// Outputs of every kernel are fully reduced, so results are canonical.
#include "gpu.h"

namespace gpu {

typedef uint64_t u64;

#define DEV __device__ __forceinline__

DEV u64 add_mod(u64 a, u64 b, u64 q) {
    u64 s = a + b;
    return s >= q ? s - q : s;
}
DEV u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
DEV u64 mul_shoup(u64 a, u64 w, u64 wsh, u64 q) {
    u64 h = __umul64hi(a, wsh);
    u64 r = a * w - h * q;
    return r >= q ? r - q : r;
}
// x = hi:lo < q^2
DEV u64 barrett(u64 hi, u64 lo, const DevPrime &P) {
    const uint32_t n = P.nbits;
    u64 t = (hi << (65 - n)) | (lo >> (n - 1));
    u64 ph = __umul64hi(t, P.mu), pl = t * P.mu;
    u64 qh = (ph << (63 - n)) | (pl >> (n + 1));
    u64 r = lo - qh * P.q;
    if (r >= P.q) r -= P.q;
    if (r >= P.q) r -= P.q;
    return r;
}
DEV u64 mul_mod(u64 a, u64 b, const DevPrime &P) { return barrett(__umul64hi(a, b), a * b, P); }
// any x = x1:x0 < 2^128
DEV u64 reduce128(u64 x1, u64 x0, const DevPrime &P) {
    u64 ah = __umul64hi(x0, P.mu2_lo);
    u64 bl = x0 * P.mu2_hi, bh = __umul64hi(x0, P.mu2_hi);
    u64 cl = x1 * P.mu2_lo, ch = __umul64hi(x1, P.mu2_lo);
    u64 dl = x1 * P.mu2_hi;
    u64 s1 = bl + cl;
    u64 c1 = s1 < bl;
    u64 s2 = s1 + ah;
    u64 c2 = s2 < s1;
    u64 qh = dl + bh + ch + c1 + c2;
    u64 r = x0 - qh * P.q;
    if (r >= P.q) r -= P.q;
    if (r >= P.q) r -= P.q;
    return r;
}
// a 64-bit value (any) reduced mod q
DEV u64 reduce64(u64 x, const DevPrime &P) { return reduce128(0, x, P); }
DEV void mac128(u64 &hi, u64 &lo, u64 a, u64 b) {
    u64 pl = a * b, ph = __umul64hi(a, b);
    lo += pl;
    hi += ph + (lo < pl);
}

// ---------------------------------------------------------------------------
// NTT
// ---------------------------------------------------------------------------
constexpr int kTile = 4096;
constexpr int kThreads = 256;

// Contiguous pass: forward stages s in [s_lo, logN) or inverse stages with
// half-distance t = 1 .. t_end/2, on tiles of `ts` consecutive words.
template <bool INV>
__global__ void __launch_bounds__(kThreads) k_ntt_contig(u64 *data, int logN, int ts, int s_lo,
                                                         int t_end, int nlimb, LimbMap m, Tables T,
                                                         int scale_out) {
    __shared__ u64 tile[kTile];
    const int limb = blockIdx.y;
    const int pi = m.p[limb % nlimb];
    const DevPrime P = T.primes[pi];
    const u64 q = P.q;
    const size_t N = (size_t)1 << logN;
    u64 *base = data + (size_t)limb * N + (size_t)blockIdx.x * ts;
    const int g0 = blockIdx.x * ts;
    for (int i = threadIdx.x; i < ts; i += kThreads) tile[i] = base[i];
    __syncthreads();
    const int half = ts >> 1;
    if (!INV) {
        const u64 *W = T.fw + (size_t)pi * N, *Ws = T.fw_sh + (size_t)pi * N;
        for (int s = s_lo; s < logN; ++s) {
            const int lt = logN - s - 1;   // t = 2^lt
            const int t = 1 << lt;
            for (int b = threadIdx.x; b < half; b += kThreads) {
                int j = ((b >> lt) << (lt + 1)) | (b & (t - 1));
                int J = g0 + j;
                int wi = (1 << s) + (J >> (logN - s));
                u64 U = tile[j];
                u64 V = mul_shoup(tile[j + t], W[wi], Ws[wi], q);
                tile[j] = add_mod(U, V, q);
                tile[j + t] = sub_mod(U, V, q);
            }
            __syncthreads();
        }
    } else {
        const u64 *W = T.iw + (size_t)pi * N, *Ws = T.iw_sh + (size_t)pi * N;
        for (int lt = 0; (1 << lt) < t_end; ++lt) {
            const int t = 1 << lt;
            for (int b = threadIdx.x; b < half; b += kThreads) {
                int j = ((b >> lt) << (lt + 1)) | (b & (t - 1));
                int J = g0 + j;
                int wi = (int)(N >> (lt + 1)) + (J >> (lt + 1));
                u64 U = tile[j], V = tile[j + t];
                tile[j] = add_mod(U, V, q);
                tile[j + t] = mul_shoup(sub_mod(U, V, q), W[wi], Ws[wi], q);
            }
            __syncthreads();
        }
    }
    if (scale_out) {
        const u64 ni = T.ninv[pi], nis = T.ninv_sh[pi];
        for (int i = threadIdx.x; i < ts; i += kThreads) base[i] = mul_shoup(tile[i], ni, nis, q);
    } else {
        for (int i = threadIdx.x; i < ts; i += kThreads) base[i] = tile[i];
    }
}

// Strided pass over R = 2^a rows of stride B = N / R, C = kTile / R columns
// per block: forward stages 0..a-1 or inverse row half-distances 1..R/2.
template <bool INV>
__global__ void __launch_bounds__(kThreads) k_ntt_strided(u64 *data, int logN, int a, int nlimb,
                                                          LimbMap m, Tables T, int scale_out) {
    __shared__ u64 tile[kTile];
    const int limb = blockIdx.y;
    const int pi = m.p[limb % nlimb];
    const DevPrime P = T.primes[pi];
    const u64 q = P.q;
    const size_t N = (size_t)1 << logN;
    const int R = 1 << a;
    const int lc = 12 - a;             // log C
    const int C = 1 << lc;
    const int B = (int)(N >> a);
    u64 *base = data + (size_t)limb * N;
    const int r0 = blockIdx.x * C;
    for (int i = threadIdx.x; i < kTile; i += kThreads) {
        int k = i >> lc, c = i & (C - 1);
        tile[i] = base[(size_t)k * B + r0 + c];
    }
    __syncthreads();
    if (!INV) {
        const u64 *W = T.fw + (size_t)pi * N, *Ws = T.fw_sh + (size_t)pi * N;
        for (int s = 0; s < a; ++s) {
            const int lth = a - s - 1;
            const int th = 1 << lth;
            for (int b = threadIdx.x; b < kTile / 2; b += kThreads) {
                int c = b & (C - 1), p = b >> lc;
                int k = ((p >> lth) << (lth + 1)) | (p & (th - 1));
                int wi = (1 << s) + (k >> (a - s));
                int i0 = (k << lc) + c, i1 = ((k + th) << lc) + c;
                u64 U = tile[i0];
                u64 V = mul_shoup(tile[i1], W[wi], Ws[wi], q);
                tile[i0] = add_mod(U, V, q);
                tile[i1] = sub_mod(U, V, q);
            }
            __syncthreads();
        }
    } else {
        const u64 *W = T.iw + (size_t)pi * N, *Ws = T.iw_sh + (size_t)pi * N;
        for (int lth = 0; lth < a; ++lth) {
            const int th = 1 << lth;
            for (int b = threadIdx.x; b < kTile / 2; b += kThreads) {
                int c = b & (C - 1), p = b >> lc;
                int k = ((p >> lth) << (lth + 1)) | (p & (th - 1));
                int wi = (R >> (lth + 1)) + (k >> (lth + 1));
                int i0 = (k << lc) + c, i1 = ((k + th) << lc) + c;
                u64 U = tile[i0], V = tile[i1];
                tile[i0] = add_mod(U, V, q);
                tile[i1] = mul_shoup(sub_mod(U, V, q), W[wi], Ws[wi], q);
            }
            __syncthreads();
        }
    }
    const u64 ni = T.ninv[pi], nis = T.ninv_sh[pi];
    for (int i = threadIdx.x; i < kTile; i += kThreads) {
        int k = i >> lc, c = i & (C - 1);
        u64 v = tile[i];
        if (scale_out) v = mul_shoup(v, ni, nis, q);
        base[(size_t)k * B + r0 + c] = v;
    }
}

// centred lift of a word mod q_top to the prime of index pi (rescale, ModRaise)
struct Lifter {
    u64 half, qt_mod;
    DevPrime P;
    DEV Lifter(const Tables &T, int top, int pi) : P(T.primes[pi]) {
        const u64 qt = T.primes[top].q;
        half = (qt - 1) >> 1;
        qt_mod = reduce64(qt, P);
    }
    DEV u64 operator()(u64 v) const {
        const u64 r = reduce64(v, P);
        return v > half ? sub_mod(r, qt_mod, P.q) : r;
    }
};
// epilogue of a fused forward transform: (c - x) * inv mod q
DEV u64 epi_word(u64 x, u64 c, u64 iv, u64 ivs, u64 q) { return mul_shoup(sub_mod(c, x, q), iv, ivs, q); }
// the epilogue's added term for poly pidx, limb lidx, tile offset off (null if none)
DEV const u64 *epi_add_ptr(const NttEpi &ep, uint32_t pidx, uint32_t lidx, size_t row_off, size_t off) {
    if (!ep.add || !((ep.add_mask >> (pidx & 1)) & 1)) return nullptr;
    if (ep.add_stride) return ep.add + (size_t)pidx * ep.add_stride + ((size_t)lidx << 16) + off;
    return ep.add + row_off + off;
}

// ---------------------------------------------------------------------------
// N = 2^16: two passes of 8 stages, each split into two radix-16 register
// phases (4 butterfly stages on 16 words held by one thread) around one LDS
// transpose.  Pass "rows": a block owns C = 16 consecutive columns of the
// 256 x 256 view (element (k, c) at k*256 + c); pass "blocks": a block owns
// 16 consecutive 256-word blocks.  256 threads, thread t -> (x = t & 15,
// y = t >> 4).  Global accesses are 16 consecutive words per 16 threads.
// ---------------------------------------------------------------------------
constexpr int kPad = 17;   // LDS row pitch (words) for the 16-wide sub-tiles

// Lazy (Harvey) butterflies for the N = 2^16 passes (primes q < 2^61): the
// products are Shoup products with a truncated quotient (below), which lie in
// [0, 4q) for any 64-bit input; values are reduced to [0, q) only where a
// transform writes its final output.
// x mod q for any 64-bit x: Shoup product by 1 (quotient constant floor(2^64/q)),
// which lands in [0, 2q), then one correction
DEV u64 reduce_any(u64 x, u64 inv64, u64 q) {
    u64 r = x - __umul64hi(x, inv64) * q;
    return r >= q ? r - q : r;
}
// Shoup product with a truncated quotient: of the four 32 x 32 partial products
// of a * wsh only the high words of the three upper ones are kept, so the
// quotient is short by at most 2 and the result lies in [0, 4q) for any 64-bit
// a (three multiplications fewer than the exact high word).
DEV u64 mul_shoup_lazy4(u64 a, u64 w, u64 wsh, u64 q) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t s0 = (uint32_t)wsh, s1 = (uint32_t)(wsh >> 32);
    const u64 Q = (u64)a1 * s1 + __umulhi(a1, s0) + __umulhi(a0, s1);
    return a * w - Q * q;
}
// Forward (CT) butterflies: U + V and U - V + 4q with V in [0, 4q).  Primes
// below 2^57 leave headroom for all 16 stages with no reduction: each stage
// adds at most 4q to the bound, so a transform from [0, q) ends below 65 q <
// 2^64.  For larger primes (q < 2^61) U is first brought into [0, 4q) by one
// conditional subtraction, which keeps every value below 8q < 2^64.  Inverse
// (GS) butterflies keep every value in [0, 4q) for every prime: S = U + V
// corrected by 4q, D = U - V + 4q < 8q into the product.
constexpr u64 kSmallPrime = 1ull << 57;

// Binary64 butterflies for primes q < 2^42 (T.fp_bits), in the 4- and 8-word
// forms (k_nttr_*); the 16-word kernels keep every prime on the integer path,
// whose registers already set their occupancy.  A residue is held as
// an integer-valued double (exact below 2^53).  The product r = V w mod q
// (up to a multiple of q) with the twiddle w < q and wq = fl(w / q):
//   h = fl(V w), l = V w - h exactly (one FMA: the error-free product),
//   k = nearest integer to V wq (FMA against 1.5 2^52, exact rounding for
//       |V wq| < 2^51), r = fma(-k, q, h) + l.
// For |V| <= 2^50: |V wq - V w / q| <= |V| 2^-54 <= 1/16, so |r| <= 0.57 q;
// h - k q = r - l with |l| <= 2^(49+42-53) and |r| < q is below 2^53, so the
// FMA is exact, and r (an integer below 2^53) is exact.  Forward (CT)
// butterflies U + r, U - r from [0, q) grow by at most 0.57 q per stage:
// below 10 q < 2^46 after all 16 stages, no reduction needed.  Inverse (GS)
// butterflies U + V, (U - V) w double the bound per stage: below 2^8 q <
// 2^50 after a pass of 8; the second pass re-centres its input first.
constexpr double kRound = 6755399441055744.0;   // 1.5 * 2^52
DEV double fp_mulmod(double v, double w, double wq, double q) {
    const double h = v * w;
    const double l = __fma_rn(v, w, -h);
    const double k = __fma_rn(v, wq, kRound) - kRound;
    return __fma_rn(-k, q, h) + l;
}
// x - q round(x / q): the representative in about [-q/2, q/2] (|x| < 2^51)
DEV double fp_centre(double x, double q, double qinv) {
    const double k = __fma_rn(x, qinv, kRound) - kRound;
    return __fma_rn(-k, q, x);
}
// canonical residue in [0, q) as a word
DEV u64 fp_canon(double x, double q, double qinv) {
    double r = fp_centre(x, q, qinv);
    r = r < 0.0 ? r + q : r;
    return (u64)r;
}
DEV double fp_bits(u64 w) { return __longlong_as_double((long long)w); }
DEV u64 fp_word(double x) { return (u64)__double_as_longlong(x); }
DEV bool fp_prime(const Tables &T, u64 q) { return T.fp_bits > 0 && q < (1ull << T.fp_bits); }

// forward butterflies (CT) on v[0..15] for 4 stages; element m pairs with
// m + h (h = 8, 4, 2, 1); twiddle index for stage j (0..3): base_j + (m >> (4 - j))
template <bool SMALL>
__device__ __forceinline__ void fwd16(u64 v[16], const u64 *W, const u64 *Ws, int s0, int hi_part, u64 q) {
    // stage j: global stage s = s0 + j; twiddle index = 2^s + hi_part * 2^j + (m >> (4 - j))
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int h = 8 >> j;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            if (m & h) continue;
            const int wi = (1 << (s0 + j)) + (hi_part << j) + (m >> (4 - j));
            if (SMALL) {
                const u64 q4 = 4 * q;
                const u64 U = v[m];
                const u64 V = mul_shoup_lazy4(v[m + h], W[wi], Ws[wi], q);   // [0, 4q)
                v[m] = U + V;
                v[m + h] = U - V + q4;
            } else {
                const u64 q4 = 4 * q;
                const u64 U = v[m] >= q4 ? v[m] - q4 : v[m];                // [0, 4q)
                const u64 V = mul_shoup_lazy4(v[m + h], W[wi], Ws[wi], q);  // [0, 4q)
                v[m] = U + V;                                               // [0, 8q)
                v[m + h] = U - V + q4;                                      // (0, 8q)
            }
        }
    }
}
// inverse butterflies (GS) on v[0..15], distances h = 1, 2, 4, 8; group index
// for distance h: hi_part * (16 / 2h) + (m >> (log2 h + 1)); twiddle index =
// n_groups_total + group, with n_groups_total = N / (2 t_global).  Values stay
// in [0, 4q).
__device__ __forceinline__ void inv16(u64 v[16], const u64 *W, const u64 *Ws, int logN, int lt0, int hi_part,
                                      u64 q) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int h = 1 << j;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            if (m & h) continue;
            const int lt = lt0 + j;   // log2 of the global half-distance
            const int wi = (1 << (logN - lt - 1)) + (hi_part << (3 - j)) + (m >> (j + 1));
            const u64 B = 4 * q;
            const u64 U = v[m], V = v[m + h];                        // [0, 4q)
            const u64 S = U + V;
            v[m] = S >= B ? S - B : S;                               // [0, 4q)
            v[m + h] = mul_shoup_lazy4(U - V + B, W[wi], Ws[wi], q);   // [0, 4q)
        }
    }
}

// forward pass over rows (stages 0..7): reads src, writes dst
// Grid of the N = 2^16 passes: blockIdx.x = 4096-word tile, blockIdx.y =
// limb * npoly + poly (prime-major), so the same tile of the same prime for
// consecutive polys runs on the same XCD and its twiddles come from L2.
#define NTT16_INDEX(nlimb, npoly)                                                \
    const uint32_t y_ = blockIdx.y;                                           \
    const uint32_t lidx = y_ / (uint32_t)(npoly);                             \
    const uint32_t pidx = y_ - lidx * (uint32_t)(npoly);                      \
    const size_t row_off = ((size_t)pidx * (uint32_t)(nlimb) + lidx) << 16;

// The 16-word blocks passes keep each 256-word block's words among its own 16
// threads (a quarter wave), so their LDS exchanges need only the wave's own
// order (fences at wavefront scope), not a workgroup barrier.
__device__ __forceinline__ void ntt16_block_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool LIFT>
__global__ void __launch_bounds__(256) k_ntt16_rows_fwd(u64 *dst, const u64 *src, size_t src_stride, int nlimb,
                                                         int npoly, LimbMap m, Tables T, NttLift lf) {
    __shared__ u64 tile[256 * kPad];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.fw + ((size_t)pi << 16), *Ws = T.fw_sh + ((size_t)pi << 16);
    const u64 *in = LIFT ? lf.t + (size_t)pidx * lf.t_stride : src + (size_t)pidx * src_stride + ((size_t)lidx << 16);
    u64 *out = dst + row_off;
    const int c0 = blockIdx.x * 16;
    const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
    u64 v[16];
    // phase 1: rows k = y + 16 m, column x; stages 0..3 (row distances 128..16)
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = in[((y + 16 * mm) << 8) + c0 + x];
    if (LIFT) {
        const Lifter L(T, lf.top, pi);
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) v[mm] = L(v[mm]);
    }
    const bool small = q < kSmallPrime;
    if (small) fwd16<true>(v, W, Ws, 0, 0, q);
    else fwd16<false>(v, W, Ws, 0, 0, q);
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) tile[(y + 16 * mm) * kPad + x] = v[mm];
    __syncthreads();
    // phase 2: rows k = 16 y + m, column x; stages 4..7 (distances 8..1)
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = tile[(16 * y + mm) * kPad + x];
    // twiddle index 2^s + (k >> (8 - s)), k = 16 y + m: hi_part = y
    if (small) fwd16<true>(v, W, Ws, 4, y, q);
    else fwd16<false>(v, W, Ws, 4, y, q);
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) out[((16 * y + mm) << 8) + c0 + x] = v[mm];
}

// forward pass over 256-word blocks (stages 8..15), in place
template <bool EPI>
__global__ void __launch_bounds__(256) k_ntt16_blocks_fwd(u64 *data, int nlimb, int npoly, LimbMap m, Tables T,
                                                           NttEpi ep) {
    __shared__ u64 tile[256 * kPad];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.fw + ((size_t)pi << 16), *Ws = T.fw_sh + ((size_t)pi << 16);
    u64 *d = data + row_off + ((size_t)blockIdx.x << 12);
    const int blk0 = blockIdx.x * 16;   // global index of the first 256-block
    const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
    u64 v[16];
    // phase 1: block y, words x + 16 m; stages 8..11 (distances 128..16)
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = d[(y << 8) + x + 16 * mm];
    // twiddle 2^s + (J >> (16 - s)), J = 256 (blk0 + y) + x + 16 m: hi_part = blk0 + y
    const bool small = q < kSmallPrime;
    if (small) fwd16<true>(v, W, Ws, 8, blk0 + y, q);
    else fwd16<false>(v, W, Ws, 8, blk0 + y, q);
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) tile[(y * 16 + mm) * kPad + x] = v[mm];   // [block y][row mm][col x]
    ntt16_block_sync();
    // phase 2: block y, words 16 x + m; stages 12..15 (distances 8..1)
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = tile[(y * 16 + x) * kPad + mm];
    if (small) {
        fwd16<true>(v, W, Ws, 12, (blk0 + y) * 16 + x, q);
        const u64 inv64 = T.primes[pi].mu2_hi;
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) v[mm] = reduce_any(v[mm], inv64, q);
    } else {
        fwd16<false>(v, W, Ws, 12, (blk0 + y) * 16 + x, q);
        const u64 inv64 = T.primes[pi].mu2_hi;
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) v[mm] = reduce_any(v[mm], inv64, q);
    }
    ntt16_block_sync();
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) tile[(y * 16 + x) * kPad + mm] = v[mm];
    ntt16_block_sync();
    if (EPI) {
        const size_t off = ((size_t)blockIdx.x << 12);
        const u64 *cc = ep.c + (size_t)pidx * ep.c_stride + ((size_t)lidx << 16) + off;
        u64 *o = ep.out + row_off + off;
        const u64 iv = ep.inv[lidx], ivs = ep.inv_sh[lidx];
        const u64 *ad = epi_add_ptr(ep, pidx, lidx, row_off, off);
        const u64 aw = ep.add_w ? ep.add_w[lidx] : 0, aws = ep.add_w ? ep.add_wsh[lidx] : 0;
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) {
            const int at = (y << 8) + x + 16 * mm;
            const u64 r = epi_word(tile[(y * 16 + mm) * kPad + x], cc[at], iv, ivs, q);
            o[at] = ad ? add_mod(r, ep.add_w ? mul_shoup(ad[at], aw, aws, q) : ad[at], q) : r;
        }
    } else {
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) d[(y << 8) + x + 16 * mm] = tile[(y * 16 + mm) * kPad + x];
    }
}

// inverse pass over 256-word blocks (half-distances 1..128): reads src, writes dst
__global__ void __launch_bounds__(256) k_ntt16_blocks_inv(u64 *dst, const u64 *src, size_t src_stride, int nlimb,
                                                           int npoly, LimbMap m, Tables T) {
    __shared__ u64 tile[256 * kPad];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.iw + ((size_t)pi << 16), *Ws = T.iw_sh + ((size_t)pi << 16);
    const u64 *s_in = src + (size_t)pidx * src_stride + ((size_t)lidx << 16) + ((size_t)blockIdx.x << 12);
    u64 *d = dst + row_off + ((size_t)blockIdx.x << 12);
    const int blk0 = blockIdx.x * 16;
    const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
    u64 v[16];
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) tile[(y * 16 + mm) * kPad + x] = s_in[(y << 8) + x + 16 * mm];
    ntt16_block_sync();
    // phase A: block y, words 16 x + m; half-distances 1..8.  Group index of
    // word J for distance t: J >> (lt + 1), J = 256 (blk0 + y) + 16 x + m
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = tile[(y * 16 + x) * kPad + mm];
    inv16(v, W, Ws, 16, 0, (blk0 + y) * 16 + x, q);
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) tile[(y * 16 + x) * kPad + mm] = v[mm];
    ntt16_block_sync();
    // phase B: block y, words x + 16 m; half-distances 16..128
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = tile[(y * 16 + mm) * kPad + x];
    inv16(v, W, Ws, 16, 4, blk0 + y, q);
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) d[(y << 8) + x + 16 * mm] = v[mm];
}

// inverse pass over rows (half-distances 256..32768, row distances 1..128), in
// place, with the final multiplication by N^-1
__global__ void __launch_bounds__(256) k_ntt16_rows_inv(u64 *data, int nlimb, int npoly, LimbMap m, Tables T) {
    __shared__ u64 tile[256 * kPad];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.iw + ((size_t)pi << 16), *Ws = T.iw_sh + ((size_t)pi << 16);
    u64 *d = data + row_off;
    const int c0 = blockIdx.x * 16;
    const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
    u64 v[16];
    // phase A: rows k = 16 y + m (row distances 1..8 = global 256..2048)
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = d[((16 * y + mm) << 8) + c0 + x];
    inv16(v, W, Ws, 16, 8, y, q);
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) tile[(16 * y + mm) * kPad + x] = v[mm];
    __syncthreads();
    // phase B: rows k = y + 16 m (row distances 16..128)
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) v[mm] = tile[(y + 16 * mm) * kPad + x];
    inv16(v, W, Ws, 16, 12, 0, q);
    const u64 ni = T.ninv[pi], nis = T.ninv_sh[pi];
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) d[((y + 16 * mm) << 8) + c0 + x] = mul_shoup(v[mm], ni, nis, q);
}

// ---------------------------------------------------------------------------
// N = 2^16 passes with R = 4 or 8 words per thread.  Same two passes as above,
// on tiles of S independent 256-point sub-transforms ("lanes": S columns of
// the 256 x 256 view, or S blocks of 256 words; S = 16 or 4), each shared by
// 256 / R threads, so a tile takes S 256 / R threads and every wave carries a
// shorter chain of dependent work: more waves in flight when a call covers few
// limbs, and with S = 4 four times as many blocks spread over the CUs.  Tiles
// are ordered so that 8 consecutive ones run on one XCD (workgroups go to the
// XCDs round robin): the rows pass's narrow column tiles then share their
// cache lines in one L2.  Phase p holds the r = log2(R) bits
// [lo, lo + r) of the 8-bit index k within the sub-transform in registers (the
// thread supplies the other 8 - r bits) and runs the stages of the phase's
// bits; phases exchange through LDS.  Forward passes take the bits from the
// top (the last phase may repeat bits already done), inverse passes from the
// bottom.  Twiddle indices follow from the global word index J: forward stage
// s pairs J and J + 2^(15 - s) with twiddle 2^s + (J >> (16 - s)); inverse
// half-distance 2^t uses 2^(15 - t) + (J >> (t + 1)).
// ---------------------------------------------------------------------------
template <int R> struct Geo {
    static constexpr int r = R == 4 ? 2 : 3;
    static constexpr int T = 256 / R;         // threads per sub-transform
    static constexpr int NPH = (8 + r - 1) / r;
    static constexpr int tb = 8 - r;          // thread bits of k
};
// tile of block bx among nt tiles (nt a multiple of 8): consecutive tiles on one XCD
__device__ __forceinline__ int xcd_tile(int bx, int nt) { return (bx & 7) * (nt >> 3) + (bx >> 3); }
// register bits [lo, lo + r) of phase p; stage bits [s_lo, s_hi)
template <int R> __device__ constexpr int fwd_lo(int p) {
    return 8 - Geo<R>::r * (p + 1) > 0 ? 8 - Geo<R>::r * (p + 1) : 0;
}
template <int R> __device__ constexpr int inv_lo(int p) {
    return Geo<R>::r * p < 8 - Geo<R>::r ? Geo<R>::r * p : 8 - Geo<R>::r;
}
// k of register m for thread sub-index u when the register bits start at lo
template <int R> __device__ __forceinline__ int k_of(int u, int m, int lo) {
    return ((u >> lo) << (lo + Geo<R>::r)) | (m << lo) | (u & ((1 << lo) - 1));
}
// LDS address of (lane, k): rows view [k][lane] with pitch S + 1, blocks
// view [lane][k >> 4][k & 15] with pitch 17 per 16 words (256 (S + 1) words
// hold either)
template <bool ROWS, int S> __device__ __forceinline__ int lds_at(int lane, int k) {
    return ROWS ? k * (S + 1) + lane : (lane * 16 + (k >> 4)) * kPad + (k & 15);
}

// forward butterflies of stage bit b (global stage s) on registers pairing
// m and m + 2^j, j = b - lo; the twiddle index comes from J of the lower word
template <int R, bool ROWS, bool SMALL>
__device__ __forceinline__ void fwd_stage(u64 *v, int u, int lo, int b, int blkg, const u64 *W, const u64 *Ws,
                                          u64 q) {
    const int j = b - lo;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if (m & (1 << j)) continue;
        const int k = k_of<R>(u, m, lo);
        const int wi = ROWS ? (1 << (7 - b)) + (k >> (b + 1))
                            : (1 << (15 - b)) + (blkg << (7 - b)) + (k >> (b + 1));
        const int h = 1 << j;
        if (SMALL) {
            const u64 U = v[m];
            const u64 V = mul_shoup_lazy4(v[m + h], W[wi], Ws[wi], q);
            v[m] = U + V;
            v[m + h] = U - V + 4 * q;
        } else {
            const u64 q4 = 4 * q;
            const u64 U = v[m] >= q4 ? v[m] - q4 : v[m];
            const u64 V = mul_shoup_lazy4(v[m + h], W[wi], Ws[wi], q);
            v[m] = U + V;
            v[m + h] = U - V + q4;
        }
    }
}
template <int R, bool ROWS, bool SMALL>
__device__ __forceinline__ void inv_stage(u64 *v, int u, int lo, int b, int blkg, const u64 *W, const u64 *Ws,
                                          u64 q) {
    const int j = b - lo;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if (m & (1 << j)) continue;
        const int k = k_of<R>(u, m, lo);
        const int wi = ROWS ? (1 << (7 - b)) + (k >> (b + 1))
                            : (1 << (15 - b)) + (blkg << (7 - b)) + (k >> (b + 1));
        const int h = 1 << j;
        const u64 B = 4 * q;
        const u64 U = v[m], V = v[m + h];
        const u64 S = U + V;
        v[m] = S >= B ? S - B : S;
        v[m + h] = mul_shoup_lazy4(U - V + B, W[wi], Ws[wi], q);
    }
}

// The exchange between two phases: in the rows view the threads of one
// sub-transform are spread over the workgroup's waves (a workgroup barrier);
// in the blocks view a sub-transform's 256 / R <= 64 threads are one wave or
// half of one, so its LDS words are written and read by that wave alone and
// the wave's own order suffices (the wavefront-scope fences keep the
// compiler from moving the reads above the writes).
template <bool ROWS> __device__ __forceinline__ void phase_sync() {
    if (ROWS) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// binary64 twins of fwd_stage / inv_stage (bounds as stated with fp_mulmod)
template <int R, bool ROWS>
__device__ __forceinline__ void fwd_stage_fp(double *v, int u, int lo, int b, int blkg, const double *W,
                                             const double *Wq, double q) {
    const int j = b - lo;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if (m & (1 << j)) continue;
        const int k = k_of<R>(u, m, lo);
        const int wi = ROWS ? (1 << (7 - b)) + (k >> (b + 1))
                            : (1 << (15 - b)) + (blkg << (7 - b)) + (k >> (b + 1));
        const int h = 1 << j;
        const double U = v[m];
        const double r = fp_mulmod(v[m + h], W[wi], Wq[wi], q);
        v[m] = U + r;
        v[m + h] = U - r;
    }
}
template <int R, bool ROWS>
__device__ __forceinline__ void inv_stage_fp(double *v, int u, int lo, int b, int blkg, const double *W,
                                             const double *Wq, double q) {
    const int j = b - lo;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if (m & (1 << j)) continue;
        const int k = k_of<R>(u, m, lo);
        const int wi = ROWS ? (1 << (7 - b)) + (k >> (b + 1))
                            : (1 << (15 - b)) + (blkg << (7 - b)) + (k >> (b + 1));
        const int h = 1 << j;
        const double U = v[m], V = v[m + h];
        v[m] = U + V;
        v[m + h] = fp_mulmod(U - V, W[wi], Wq[wi], q);
    }
}
// binary64 twin of pass_phases (LDS exchanges carry the doubles' bits)
template <int R, int S, bool ROWS, bool FWD>
__device__ __forceinline__ void pass_phases_fp(double *v, u64 *tile, int lane, int u, int blkg, const double *W,
                                               const double *Wq, double q) {
    constexpr int r = Geo<R>::r, NPH = Geo<R>::NPH;
#pragma unroll
    for (int p = 0; p < NPH; ++p) {
        const int lo = FWD ? fwd_lo<R>(p) : inv_lo<R>(p);
        if (p > 0) {
            phase_sync<ROWS>();
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = fp_bits(tile[lds_at<ROWS, S>(lane, k_of<R>(u, m, lo))]);
        }
        if (FWD) {
            const int b_hi = 8 - r * p - 1, b_lo = lo;
#pragma unroll
            for (int b = b_hi; b >= b_lo; --b) fwd_stage_fp<R, ROWS>(v, u, lo, b, blkg, W, Wq, q);
        } else {
            const int b_lo = r * p, b_hi = (r * (p + 1) < 8 ? r * (p + 1) : 8) - 1;
#pragma unroll
            for (int b = b_lo; b <= b_hi; ++b) inv_stage_fp<R, ROWS>(v, u, lo, b, blkg, W, Wq, q);
        }
        if (p + 1 < NPH) {
#pragma unroll
            for (int m = 0; m < R; ++m) tile[lds_at<ROWS, S>(lane, k_of<R>(u, m, lo))] = fp_word(v[m]);
        }
    }
}

// all phases of one pass on registers v (loaded for phase 0 by the caller);
// leaves the registers holding the last phase's words
template <int R, int S, bool ROWS, bool FWD, bool SMALL>
__device__ __forceinline__ void pass_phases(u64 *v, u64 *tile, int lane, int u, int blkg, const u64 *W,
                                            const u64 *Ws, u64 q) {
    constexpr int r = Geo<R>::r, NPH = Geo<R>::NPH;
#pragma unroll
    for (int p = 0; p < NPH; ++p) {
        const int lo = FWD ? fwd_lo<R>(p) : inv_lo<R>(p);
        if (p > 0) {
            phase_sync<ROWS>();   // the previous phase's words are all in LDS
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = tile[lds_at<ROWS, S>(lane, k_of<R>(u, m, lo))];
        }
        if (FWD) {
            const int b_hi = 8 - r * p - 1, b_lo = lo;   // stage bits, high to low
#pragma unroll
            for (int b = b_hi; b >= b_lo; --b) fwd_stage<R, ROWS, SMALL>(v, u, lo, b, blkg, W, Ws, q);
        } else {
            const int b_lo = r * p, b_hi = (r * (p + 1) < 8 ? r * (p + 1) : 8) - 1;
#pragma unroll
            for (int b = b_lo; b <= b_hi; ++b) inv_stage<R, ROWS, SMALL>(v, u, lo, b, blkg, W, Ws, q);
        }
        if (p + 1 < NPH) {
            // each thread writes back exactly the words it read in this phase
#pragma unroll
            for (int m = 0; m < R; ++m) tile[lds_at<ROWS, S>(lane, k_of<R>(u, m, lo))] = v[m];
        }
    }
}

// forward rows pass (stages 0..7): src -> dst
template <int R, int S, bool LIFT>
__global__ void __launch_bounds__(S * Geo<R>::T) k_nttr_rows_fwd(u64 *dst, const u64 *src, size_t src_stride,
                                                                  int nlimb, int npoly, LimbMap m, Tables T,
                                                                  NttLift lf) {
    __shared__ u64 tile[256 * (S + 1)];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.fw + ((size_t)pi << 16), *Ws = T.fw_sh + ((size_t)pi << 16);
    const u64 *in = LIFT ? lf.t + (size_t)pidx * lf.t_stride : src + (size_t)pidx * src_stride + ((size_t)lidx << 16);
    u64 *out = dst + row_off;
    const int c0 = xcd_tile(blockIdx.x, gridDim.x) * S;
    const int lane = threadIdx.x % S, u = threadIdx.x / S;
    constexpr int lo0 = fwd_lo<R>(0), loL = fwd_lo<R>(Geo<R>::NPH - 1);
    u64 v[R];
#pragma unroll
    for (int mm = 0; mm < R; ++mm) v[mm] = in[(k_of<R>(u, mm, lo0) << 8) + c0 + lane];
    if (LIFT) {
        const Lifter L(T, lf.top, pi);
#pragma unroll
        for (int mm = 0; mm < R; ++mm) v[mm] = L(v[mm]);
    }
    if (fp_prime(T, q)) {
        double f[R];
#pragma unroll
        for (int mm = 0; mm < R; ++mm) f[mm] = (double)v[mm];
        pass_phases_fp<R, S, true, true>(f, tile, lane, u, 0, T.fw_d + ((size_t)pi << 16),
                                         T.fwq_d + ((size_t)pi << 16), T.pd[4 * pi]);
#pragma unroll
        for (int mm = 0; mm < R; ++mm) out[(k_of<R>(u, mm, loL) << 8) + c0 + lane] = fp_word(f[mm]);
        return;
    }
    if (q < kSmallPrime) pass_phases<R, S, true, true, true>(v, tile, lane, u, 0, W, Ws, q);
    else pass_phases<R, S, true, true, false>(v, tile, lane, u, 0, W, Ws, q);
#pragma unroll
    for (int mm = 0; mm < R; ++mm) out[(k_of<R>(u, mm, loL) << 8) + c0 + lane] = v[mm];
}
// forward blocks pass (stages 8..15), in place, output reduced to [0, q)
template <int R, int S, bool EPI>
__global__ void __launch_bounds__(S * Geo<R>::T) k_nttr_blocks_fwd(u64 *data, int nlimb, int npoly, LimbMap m,
                                                                    Tables T, NttEpi ep) {
    __shared__ u64 tile[256 * (S + 1)];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.fw + ((size_t)pi << 16), *Ws = T.fw_sh + ((size_t)pi << 16);
    const int tl = xcd_tile(blockIdx.x, gridDim.x);
    const size_t off = (size_t)tl * S * 256;
    u64 *d = data + row_off + off;
    const int lane = threadIdx.x / Geo<R>::T, u = threadIdx.x % Geo<R>::T;
    const int blkg = tl * S + lane;
    constexpr int lo0 = fwd_lo<R>(0), loL = fwd_lo<R>(Geo<R>::NPH - 1);
    u64 v[R];
    if (fp_prime(T, q)) {
        const double qd = T.pd[4 * pi], qi = T.pd[4 * pi + 1];
        double f[R];
#pragma unroll
        for (int mm = 0; mm < R; ++mm) f[mm] = fp_bits(d[(lane << 8) + k_of<R>(u, mm, lo0)]);
        pass_phases_fp<R, S, false, true>(f, tile, lane, u, blkg, T.fw_d + ((size_t)pi << 16),
                                          T.fwq_d + ((size_t)pi << 16), qd);
#pragma unroll
        for (int mm = 0; mm < R; ++mm) v[mm] = fp_canon(f[mm], qd, qi);
    } else {
#pragma unroll
        for (int mm = 0; mm < R; ++mm) v[mm] = d[(lane << 8) + k_of<R>(u, mm, lo0)];
        if (q < kSmallPrime) pass_phases<R, S, false, true, true>(v, tile, lane, u, blkg, W, Ws, q);
        else pass_phases<R, S, false, true, false>(v, tile, lane, u, blkg, W, Ws, q);
        const u64 inv64 = T.primes[pi].mu2_hi;
#pragma unroll
        for (int mm = 0; mm < R; ++mm) v[mm] = reduce_any(v[mm], inv64, q);
    }
    if (EPI) {
        const u64 *cc = ep.c + (size_t)pidx * ep.c_stride + ((size_t)lidx << 16) + off;
        u64 *o = ep.out + row_off + off;
        const u64 iv = ep.inv[lidx], ivs = ep.inv_sh[lidx];
        const u64 *ad = epi_add_ptr(ep, pidx, lidx, row_off, off);
        const u64 aw = ep.add_w ? ep.add_w[lidx] : 0, aws = ep.add_w ? ep.add_wsh[lidx] : 0;
#pragma unroll
        for (int mm = 0; mm < R; ++mm) {
            const int at = (lane << 8) + k_of<R>(u, mm, loL);
            const u64 r = epi_word(v[mm], cc[at], iv, ivs, q);
            o[at] = ad ? add_mod(r, ep.add_w ? mul_shoup(ad[at], aw, aws, q) : ad[at], q) : r;
        }
    } else {
#pragma unroll
        for (int mm = 0; mm < R; ++mm) d[(lane << 8) + k_of<R>(u, mm, loL)] = v[mm];
    }
}
// inverse blocks pass (half-distances 1..128): src -> dst
template <int R, int S>
__global__ void __launch_bounds__(S * Geo<R>::T) k_nttr_blocks_inv(u64 *dst, const u64 *src, size_t src_stride,
                                                                    int nlimb, int npoly, LimbMap m, Tables T) {
    __shared__ u64 tile[256 * (S + 1)];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.iw + ((size_t)pi << 16), *Ws = T.iw_sh + ((size_t)pi << 16);
    const int tl = xcd_tile(blockIdx.x, gridDim.x);
    const size_t off = (size_t)tl * S * 256;
    const u64 *s_in = src + (size_t)pidx * src_stride + ((size_t)lidx << 16) + off;
    u64 *d = dst + row_off + off;
    const int lane = threadIdx.x / Geo<R>::T, u = threadIdx.x % Geo<R>::T;
    const int blkg = tl * S + lane;
    constexpr int lo0 = inv_lo<R>(0), loL = inv_lo<R>(Geo<R>::NPH - 1);
    u64 v[R];
#pragma unroll
    for (int mm = 0; mm < R; ++mm) v[mm] = s_in[(lane << 8) + k_of<R>(u, mm, lo0)];
    if (fp_prime(T, q)) {
        double f[R];
#pragma unroll
        for (int mm = 0; mm < R; ++mm) f[mm] = (double)v[mm];
        pass_phases_fp<R, S, false, false>(f, tile, lane, u, blkg, T.iw_d + ((size_t)pi << 16),
                                           T.iwq_d + ((size_t)pi << 16), T.pd[4 * pi]);
#pragma unroll
        for (int mm = 0; mm < R; ++mm) d[(lane << 8) + k_of<R>(u, mm, loL)] = fp_word(f[mm]);
        return;
    }
    pass_phases<R, S, false, false, true>(v, tile, lane, u, blkg, W, Ws, q);   // inverse: one path for all primes
#pragma unroll
    for (int mm = 0; mm < R; ++mm) d[(lane << 8) + k_of<R>(u, mm, loL)] = v[mm];
}
// inverse rows pass (half-distances 256..32768), in place, times N^-1
template <int R, int S>
__global__ void __launch_bounds__(S * Geo<R>::T) k_nttr_rows_inv(u64 *data, int nlimb, int npoly, LimbMap m,
                                                                  Tables T) {
    __shared__ u64 tile[256 * (S + 1)];
    NTT16_INDEX(nlimb, npoly)
    const int pi = m.p[lidx];
    const u64 q = T.primes[pi].q;
    const u64 *W = T.iw + ((size_t)pi << 16), *Ws = T.iw_sh + ((size_t)pi << 16);
    u64 *d = data + row_off;
    const int c0 = xcd_tile(blockIdx.x, gridDim.x) * S;
    const int lane = threadIdx.x % S, u = threadIdx.x / S;
    constexpr int lo0 = inv_lo<R>(0), loL = inv_lo<R>(Geo<R>::NPH - 1);
    u64 v[R];
    if (fp_prime(T, q)) {
        const double qd = T.pd[4 * pi], qi = T.pd[4 * pi + 1], nd = T.pd[4 * pi + 2], ndq = T.pd[4 * pi + 3];
        double f[R];
#pragma unroll
        for (int mm = 0; mm < R; ++mm) f[mm] = fp_centre(fp_bits(d[(k_of<R>(u, mm, lo0) << 8) + c0 + lane]), qd, qi);
        pass_phases_fp<R, S, true, false>(f, tile, lane, u, 0, T.iw_d + ((size_t)pi << 16),
                                          T.iwq_d + ((size_t)pi << 16), qd);
#pragma unroll
        for (int mm = 0; mm < R; ++mm)
            d[(k_of<R>(u, mm, loL) << 8) + c0 + lane] = fp_canon(fp_mulmod(f[mm], nd, ndq, qd), qd, qi);
        return;
    }
#pragma unroll
    for (int mm = 0; mm < R; ++mm) v[mm] = d[(k_of<R>(u, mm, lo0) << 8) + c0 + lane];
    pass_phases<R, S, true, false, true>(v, tile, lane, u, 0, W, Ws, q);   // inverse: one path for all primes
    const u64 ni = T.ninv[pi], nis = T.ninv_sh[pi];
#pragma unroll
    for (int mm = 0; mm < R; ++mm) d[(k_of<R>(u, mm, loL) << 8) + c0 + lane] = mul_shoup(v[mm], ni, nis, q);
}

template <int R, int S>
static void launch_nttr(const Tables &T, uint64_t *dst, const uint64_t *src, size_t src_poly_stride, int nlimb,
                        int npoly, const LimbMap &m, bool inverse, hipStream_t s) {
    dim3 grid(256 / S, nlimb * npoly), block(S * Geo<R>::T);
    if (!inverse) {
        k_nttr_rows_fwd<R, S, false><<<grid, block, 0, s>>>(dst, src, src_poly_stride, nlimb, npoly, m, T, NttLift{});
        k_nttr_blocks_fwd<R, S, false><<<grid, block, 0, s>>>(dst, nlimb, npoly, m, T, NttEpi{});
    } else {
        hipLaunchKernelGGL((k_nttr_blocks_inv<R, S>), grid, block, 0, s, dst, src, src_poly_stride, nlimb, npoly, m, T);
        hipLaunchKernelGGL((k_nttr_rows_inv<R, S>), grid, block, 0, s, dst, nlimb, npoly, m, T);
    }
}
template <int R, int S>
static void launch_nttr_fused(const Tables &T, uint64_t *work, const NttLift *lift, const NttEpi *epi, int nlimb,
                              int npoly, const LimbMap &m, hipStream_t s) {
    const NttLift lf = lift ? *lift : NttLift{};
    const NttEpi ep = epi ? *epi : NttEpi{};
    const size_t stride = (size_t)nlimb << 16;
    dim3 grid(256 / S, nlimb * npoly), block(S * Geo<R>::T);
    if (lift) k_nttr_rows_fwd<R, S, true><<<grid, block, 0, s>>>(work, work, stride, nlimb, npoly, m, T, lf);
    else k_nttr_rows_fwd<R, S, false><<<grid, block, 0, s>>>(work, work, stride, nlimb, npoly, m, T, lf);
    if (epi) k_nttr_blocks_fwd<R, S, true><<<grid, block, 0, s>>>(work, nlimb, npoly, m, T, ep);
    else k_nttr_blocks_fwd<R, S, false><<<grid, block, 0, s>>>(work, nlimb, npoly, m, T, ep);
}

void ntt16_fwd_fused(const Tables &T, uint64_t *work, const NttLift *lift, const NttEpi *epi, int nlimb, int npoly,
                     const LimbMap &m, hipStream_t s) {
    const int total = nlimb * npoly;
    if (total == 0 || T.logN != 16) return;
    const NttLift lf = lift ? *lift : NttLift{};
    const NttEpi ep = epi ? *epi : NttEpi{};
    const size_t stride = (size_t)nlimb << 16;
    if (total <= T.ntt_r4_max) {
        if (total <= T.ntt_s4_max) launch_nttr_fused<4, 4>(T, work, lift, epi, nlimb, npoly, m, s);
        else launch_nttr_fused<4, 16>(T, work, lift, epi, nlimb, npoly, m, s);
        return;
    }
    if (total <= T.ntt_r8_max) {
        launch_nttr_fused<8, 16>(T, work, lift, epi, nlimb, npoly, m, s);
        return;
    }
    dim3 grid(16, total);
    if (lift) k_ntt16_rows_fwd<true><<<grid, dim3(256), 0, s>>>(work, work, stride, nlimb, npoly, m, T, lf);
    else k_ntt16_rows_fwd<false><<<grid, dim3(256), 0, s>>>(work, work, stride, nlimb, npoly, m, T, lf);
    if (epi) k_ntt16_blocks_fwd<true><<<grid, dim3(256), 0, s>>>(work, nlimb, npoly, m, T, ep);
    else k_ntt16_blocks_fwd<false><<<grid, dim3(256), 0, s>>>(work, nlimb, npoly, m, T, ep);
}

void ntt_oop(const Tables &T, uint64_t *dst, const uint64_t *src, size_t src_poly_stride, int nlimb, int npoly,
             const LimbMap &m, bool inverse, hipStream_t s) {
    const int total = nlimb * npoly;
    if (total == 0) return;
    const size_t N = (size_t)1 << T.logN;
    if (src_poly_stride == 0) src_poly_stride = (size_t)nlimb * N;
    if (T.logN == 16) {
        // words per thread from the call's size (tunable per context): short
        // per-wave chains for small calls, fewer LDS exchanges for large ones
        if (total <= T.ntt_r4_max) {
            if (total <= T.ntt_s4_max) launch_nttr<4, 4>(T, dst, src, src_poly_stride, nlimb, npoly, m, inverse, s);
            else launch_nttr<4, 16>(T, dst, src, src_poly_stride, nlimb, npoly, m, inverse, s);
            return;
        }
        if (total <= T.ntt_r8_max) {
            launch_nttr<8, 16>(T, dst, src, src_poly_stride, nlimb, npoly, m, inverse, s);
            return;
        }
        dim3 grid(16, total);
        if (!inverse) {
            k_ntt16_rows_fwd<false><<<grid, dim3(256), 0, s>>>(dst, src, src_poly_stride, nlimb, npoly, m, T,
                                                               NttLift{});
            k_ntt16_blocks_fwd<false><<<grid, dim3(256), 0, s>>>(dst, nlimb, npoly, m, T, NttEpi{});
        } else {
            hipLaunchKernelGGL(k_ntt16_blocks_inv, grid, dim3(256), 0, s, dst, src, src_poly_stride, nlimb, npoly, m,
                               T);
            hipLaunchKernelGGL(k_ntt16_rows_inv, grid, dim3(256), 0, s, dst, nlimb, npoly, m, T);
        }
        return;
    }
    if (dst != src || src_poly_stride != (size_t)nlimb * N)
        for (int p = 0; p < npoly; ++p)
            (void)hipMemcpyAsync(dst + (size_t)p * nlimb * N, src + (size_t)p * src_poly_stride, (size_t)nlimb * N * 8,
                                 hipMemcpyDeviceToDevice, s);
    ntt(T, dst, nlimb, npoly, m, inverse, s);
}

void ntt(const Tables &T, uint64_t *data, int nlimb, int npoly, const LimbMap &m, bool inverse,
         hipStream_t s) {
    const int logN = T.logN;
    if (logN == 16) {
        ntt_oop(T, data, data, 0, nlimb, npoly, m, inverse, s);
        return;
    }
    const int N = 1 << logN;
    const int total = nlimb * npoly;
    if (total == 0) return;
    if (N <= kTile) {
        dim3 grid(1, total);
        if (!inverse)
            hipLaunchKernelGGL(k_ntt_contig<false>, grid, dim3(kThreads), 0, s, data, logN, N, 0, 0, nlimb, m, T, 0);
        else
            hipLaunchKernelGGL(k_ntt_contig<true>, grid, dim3(kThreads), 0, s, data, logN, N, 0, N, nlimb, m, T, 1);
        return;
    }
    const int a = 8;               // rows of the strided pass: 256
    const int b = logN - a;        // contiguous block 2^b
    dim3 gs(N / kTile, total);   // column blocks of C = kTile / 2^a columns
    dim3 gc(N / kTile, total);
    if (!inverse) {
        hipLaunchKernelGGL(k_ntt_strided<false>, gs, dim3(kThreads), 0, s, data, logN, a, nlimb, m, T, 0);
        hipLaunchKernelGGL(k_ntt_contig<false>, gc, dim3(kThreads), 0, s, data, logN, kTile, a, 0, nlimb, m, T, 0);
    } else {
        hipLaunchKernelGGL(k_ntt_contig<true>, gc, dim3(kThreads), 0, s, data, logN, kTile, 0, 1 << b, nlimb, m, T, 0);
        hipLaunchKernelGGL(k_ntt_strided<true>, gs, dim3(kThreads), 0, s, data, logN, a, nlimb, m, T, 1);
    }
}

// ---------------------------------------------------------------------------
// Elementwise kernels (grid-stride over limbs x words)
// ---------------------------------------------------------------------------
static inline dim3 grid_for(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 65535u * 8u) b = 65535u * 8u;
    return dim3((unsigned)b);
}
// row = word index >> logN (< 2^31); poly / limb split in 32-bit integer arithmetic
#define ROW_SPLIT(i, logN, nlimb, poly, limb)               \
    const uint32_t row_ = (uint32_t)((i) >> (logN));        \
    const uint32_t poly = row_ / (uint32_t)(nlimb);         \
    const uint32_t limb = row_ - poly * (uint32_t)(nlimb);
#define GRID_LOOP(idx, total) \
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (total); idx += (size_t)gridDim.x * blockDim.x)

__global__ void k_add(u64 *out, const u64 *a, const u64 *b, int logN, int nlimb, size_t total, LimbMap m,
                      Tables T, int sub) {
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        (void)poly;
        u64 q = T.primes[m.p[limb]].q;
        out[i] = sub ? sub_mod(a[i], b[i], q) : add_mod(a[i], b[i], q);
    }
}
// the same with 4 words per thread (N >= 1024; blocks of 1024 words of one row)
__global__ void __launch_bounds__(256) k_add4(u64 *out, const u64 *a, const u64 *b, int logN, int nlimb,
                                              size_t total, LimbMap m, Tables T, int sub) {
    for (size_t base = (size_t)blockIdx.x * 1024; base < total; base += (size_t)gridDim.x * 1024) {
        const uint32_t row_ = (uint32_t)(base >> logN);
        const uint32_t limb = row_ % (uint32_t)nlimb;
        const u64 q = T.primes[m.p[limb]].q;
        const size_t i0 = base + threadIdx.x;
        u64 x[4], y[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            x[e] = a[i0 + 256 * e];
            y[e] = b[i0 + 256 * e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) out[i0 + 256 * e] = sub ? sub_mod(x[e], y[e], q) : add_mod(x[e], y[e], q);
    }
}
static inline dim3 grid_for4(size_t n);
void add(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *b, int nlimb, int npoly,
         const LimbMap &m, bool sub, hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    if (T.logN >= 10) {
        hipLaunchKernelGGL(k_add4, grid_for4(total), dim3(256), 0, s, out, a, b, T.logN, nlimb, total, m, T, (int)sub);
        return;
    }
    hipLaunchKernelGGL(k_add, grid_for(total), dim3(256), 0, s, out, a, b, T.logN, nlimb, total, m, T, (int)sub);
}

__global__ void k_mul_scalar(u64 *out, const u64 *a, LimbConsts c, int logN, int nlimb, size_t total, LimbMap m,
                             Tables T) {
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        (void)poly;
        u64 q = T.primes[m.p[limb]].q;
        out[i] = mul_shoup(a[i], c.v[limb], c.sh[limb], q);
    }
}
void mul_scalar(const Tables &T, uint64_t *out, const uint64_t *a, const LimbConsts &c, int nlimb, int npoly,
                const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_mul_scalar, grid_for(total), dim3(256), 0, s, out, a, c, T.logN, nlimb, total, m, T);
}

// k a, plus the constant c on poly 0 of every member: an integer multiply and
// a constant addition in one pass
__global__ void k_mul_add_scalar(u64 *out, const u64 *a, LimbConsts k, LimbWords c, int logN, int nlimb,
                                 size_t total, LimbMap m, Tables T) {
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        const u64 q = T.primes[m.p[limb]].q;
        const u64 r = mul_shoup(a[i], k.v[limb], k.sh[limb], q);
        out[i] = (poly & 1) ? r : add_mod(r, c.v[limb], q);
    }
}
// the same with 4 words per thread (N >= 1024): a block covers 1024
// consecutive words of one row, each load instruction still coalesced, and
// the row's constants are block uniform
__global__ void __launch_bounds__(256) k_mul_add_scalar4(u64 *out, const u64 *a, LimbConsts k, LimbWords c,
                                                         int logN, int nlimb, size_t total, LimbMap m, Tables T) {
    for (size_t base = (size_t)blockIdx.x * 1024; base < total; base += (size_t)gridDim.x * 1024) {
        const uint32_t row_ = (uint32_t)(base >> logN);
        const uint32_t poly = row_ / (uint32_t)nlimb;
        const uint32_t limb = row_ - poly * (uint32_t)nlimb;
        const u64 q = T.primes[m.p[limb]].q;
        const size_t i0 = base + threadIdx.x;
        u64 x[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = a[i0 + 256 * e];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const u64 r = mul_shoup(x[e], k.v[limb], k.sh[limb], q);
            out[i0 + 256 * e] = (poly & 1) ? r : add_mod(r, c.v[limb], q);
        }
    }
}
static inline dim3 grid_for4(size_t n) {
    size_t b = (n + 1023) / 1024;
    if (b > 65535u * 8u) b = 65535u * 8u;
    return dim3((unsigned)b);
}
void mul_add_scalar(const Tables &T, uint64_t *out, const uint64_t *a, const LimbConsts &k, const LimbWords &c,
                    int nlimb, int npoly, const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    if (T.logN >= 10)
        hipLaunchKernelGGL(k_mul_add_scalar4, grid_for4(total), dim3(256), 0, s, out, a, k, c, T.logN, nlimb, total,
                           m, T);
    else
        hipLaunchKernelGGL(k_mul_add_scalar, grid_for(total), dim3(256), 0, s, out, a, k, c, T.logN, nlimb, total, m,
                           T);
}

__global__ void k_add_scalar(u64 *out, const u64 *a, LimbConsts c, int logN, int nlimb, size_t total, LimbMap m,
                             Tables T) {
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        if ((poly & 1) == 0) {
            u64 q = T.primes[m.p[limb]].q;
            out[i] = add_mod(a[i], c.v[limb], q);
        } else {
            out[i] = a[i];
        }
    }
}
void add_scalar(const Tables &T, uint64_t *out, const uint64_t *a, const LimbConsts &c, int nlimb, int npoly,
                const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_add_scalar, grid_for(total), dim3(256), 0, s, out, a, c, T.logN, nlimb, total, m, T);
}

__global__ void k_permute(u64 *out, const u64 *a, const int32_t *perm, int logN, size_t total) {
    const size_t mask = ((size_t)1 << logN) - 1;
    GRID_LOOP(i, total) {
        size_t row = i & ~mask;
        out[i] = a[row + perm[i & mask]];
    }
}
void permute(const Tables &T, uint64_t *out, const uint64_t *a, const int32_t *perm, int nlimb, int npoly,
             hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_permute, grid_for(total), dim3(256), 0, s, out, a, perm, T.logN, total);
}

__global__ void k_tensor(u64 *d01, u64 *d2, const u64 *a, const u64 *b, int logN, int nlimb, size_t total,
                         LimbMap m, Tables T) {
    const size_t per = (size_t)nlimb << logN;   // words per poly
    const size_t mask = ((size_t)1 << logN) - 1;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, ct, limb)
        const DevPrime P = T.primes[m.p[limb]];
        const size_t rem = ((size_t)limb << logN) | (i & mask);
        const size_t base = (size_t)ct * 2 * per + rem;
        u64 x0 = a[base], x1 = a[base + per], y0 = b[base], y1 = b[base + per];
        d01[base] = mul_mod(x0, y0, P);
        u64 hi = 0, lo = 0;
        mac128(hi, lo, x0, y1);
        mac128(hi, lo, x1, y0);
        d01[base + per] = reduce128(hi, lo, P);
        d2[i] = mul_mod(x1, y1, P);
    }
}
void tensor(const Tables &T, uint64_t *d01, uint64_t *d2, const uint64_t *a, const uint64_t *b, int nlimb, int nct,
            const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * nct) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_tensor, grid_for(total), dim3(256), 0, s, d01, d2, a, b, T.logN, nlimb, total, m, T);
}

__global__ void k_tensor_gather(u64 *d01, u64 *d2, GatherPtrs g, int logN, int nlimb, size_t total, LimbMap m,
                                Tables T) {
    const size_t per = (size_t)nlimb << logN;   // words per poly
    const size_t mask = ((size_t)1 << logN) - 1;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, ct, limb)
        const DevPrime P = T.primes[m.p[limb]];
        const size_t rem = ((size_t)limb << logN) | (i & mask);
        const uint32_t src = ct / (uint32_t)g.per_src, loc = ct - src * (uint32_t)g.per_src;
        const size_t sb = (size_t)loc * 2 * per + rem;
        const u64 *a = g.a[src], *b = g.b[src];
        const u64 x0 = a[sb], x1 = a[sb + per], y0 = b[sb], y1 = b[sb + per];
        const size_t base = (size_t)ct * 2 * per + rem;
        d01[base] = mul_mod(x0, y0, P);
        u64 hi = 0, lo = 0;
        mac128(hi, lo, x0, y1);
        mac128(hi, lo, x1, y0);
        d01[base + per] = reduce128(hi, lo, P);
        d2[i] = mul_mod(x1, y1, P);
    }
}
// the same with 2 words per thread (N >= 512): a block covers 512 consecutive
// words of one row, whose prime and operand pointers are block uniform
__global__ void __launch_bounds__(256) k_tensor_gather2(u64 *d01, u64 *d2, GatherPtrs g, int logN, int nlimb,
                                                        size_t total, LimbMap m, Tables T) {
    const size_t per = (size_t)nlimb << logN;
    const size_t mask = ((size_t)1 << logN) - 1;
    for (size_t base = (size_t)blockIdx.x * 512; base < total; base += (size_t)gridDim.x * 512) {
        const uint32_t row_ = (uint32_t)(base >> logN);
        const uint32_t ct = row_ / (uint32_t)nlimb;
        const uint32_t limb = row_ - ct * (uint32_t)nlimb;
        const DevPrime P = T.primes[m.p[limb]];
        const size_t rem = ((size_t)limb << logN) | ((base & mask) + threadIdx.x);
        const uint32_t src = ct / (uint32_t)g.per_src, loc = ct - src * (uint32_t)g.per_src;
        const size_t sb = (size_t)loc * 2 * per + rem;
        const u64 *a = g.a[src], *b = g.b[src];
        u64 x0[2], x1[2], y0[2], y1[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            x0[e] = a[sb + 256 * e];
            x1[e] = a[sb + per + 256 * e];
            y0[e] = b[sb + 256 * e];
            y1[e] = b[sb + per + 256 * e];
        }
        const size_t ob = (size_t)ct * 2 * per + rem;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            d01[ob + 256 * e] = mul_mod(x0[e], y0[e], P);
            u64 hi = 0, lo = 0;
            mac128(hi, lo, x0[e], y1[e]);
            mac128(hi, lo, x1[e], y0[e]);
            d01[ob + per + 256 * e] = reduce128(hi, lo, P);
            d2[base + threadIdx.x + 256 * e] = mul_mod(x1[e], y1[e], P);
        }
    }
}
void tensor_gather(const Tables &T, uint64_t *d01, uint64_t *d2, const GatherPtrs &g, int nlimb, int nct,
                   const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * nct) << T.logN;
    if (!total) return;
    if (T.logN >= 9) {
        size_t nb = (total + 511) / 512;
        if (nb > 65535u * 8u) nb = 65535u * 8u;
        hipLaunchKernelGGL(k_tensor_gather2, dim3((unsigned)nb), dim3(256), 0, s, d01, d2, g, T.logN, nlimb, total, m,
                           T);
        return;
    }
    hipLaunchKernelGGL(k_tensor_gather, grid_for(total), dim3(256), 0, s, d01, d2, g, T.logN, nlimb, total, m, T);
}

__global__ void k_mul_pointwise(u64 *out, const u64 *a, const u64 *b, int logN, int nlimb, size_t total, LimbMap m,
                                Tables T) {
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        (void)poly;
        const DevPrime P = T.primes[m.p[limb]];
        out[i] = mul_mod(a[i], b[i], P);
    }
}
void mul_pointwise(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *b, int nlimb, int npoly,
                   const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_mul_pointwise, grid_for(total), dim3(256), 0, s, out, a, b, T.logN, nlimb, total, m, T);
}

__global__ void k_mul_add(u64 *out, const u64 *a, const u64 *b, const u64 *c, int logN, size_t total, LimbMap m,
                          Tables T) {
    GRID_LOOP(i, total) {
        const DevPrime P = T.primes[m.p[i >> logN]];
        out[i] = add_mod(mul_mod(a[i], b[i], P), c[i], P.q);
    }
}
void mul_add(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *b, const uint64_t *c, int nlimb,
             const LimbMap &m, hipStream_t s) {
    size_t total = (size_t)nlimb << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_mul_add, grid_for(total), dim3(256), 0, s, out, a, b, c, T.logN, total, m, T);
}

struct Flags {
    uint8_t f[kMaxLimbs];
};
__global__ void k_key_combine(u64 *out, const u64 *a, const u64 *sk, const u64 *e, const u64 *sp, LimbConsts k,
                              Flags fl, int logN, size_t total, LimbMap m, Tables T) {
    GRID_LOOP(i, total) {
        int limb = (int)(i >> logN);
        const DevPrime P = T.primes[m.p[limb]];
        u64 v = sub_mod(e[i], mul_mod(a[i], sk[i], P), P.q);
        if (fl.f[limb]) v = add_mod(v, mul_shoup(sp[i], k.v[limb], k.sh[limb], P.q), P.q);
        out[i] = v;
    }
}
void key_combine(const Tables &T, uint64_t *out, const uint64_t *a, const uint64_t *s_, const uint64_t *e,
                 const uint64_t *sprime, const LimbConsts &k, const uint8_t *flag_host, int nlimb, const LimbMap &m,
                 hipStream_t s) {
    Flags fl;
    for (int i = 0; i < kMaxLimbs; ++i) fl.f[i] = (i < nlimb && flag_host) ? flag_host[i] : 0;
    size_t total = (size_t)nlimb << T.logN;
    hipLaunchKernelGGL(k_key_combine, grid_for(total), dim3(256), 0, s, out, a, s_, e, sprime, k, fl, T.logN, total,
                       m, T);
}

__global__ void k_signed(u64 *out, const int64_t *src, int logN, size_t total, LimbMap m, Tables T) {
    const size_t mask = ((size_t)1 << logN) - 1;
    GRID_LOOP(i, total) {
        const DevPrime P = T.primes[m.p[i >> logN]];
        int64_t v = src[i & mask];
        u64 mag = v < 0 ? (u64)(-(v + 1)) + 1 : (u64)v;
        u64 r = reduce64(mag, P);
        out[i] = (v < 0 && r) ? P.q - r : r;
    }
}
void signed_to_residues(const Tables &T, uint64_t *out, const int64_t *src, int nlimb, const LimbMap &m,
                        hipStream_t s) {
    size_t total = (size_t)nlimb << T.logN;
    hipLaunchKernelGGL(k_signed, grid_for(total), dim3(256), 0, s, out, src, T.logN, total, m, T);
}

// ---------------------------------------------------------------------------
// Rescale helpers
// ---------------------------------------------------------------------------
__global__ void k_rescale_lift(u64 *u, const u64 *t, int top, int logN, int nlimb, size_t total,
                               size_t t_stride, Tables T) {
    const size_t N = (size_t)1 << logN;
    const DevPrime Pt = T.primes[top];
    const u64 half = (Pt.q - 1) >> 1;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        const size_t j = i & (N - 1);
        const DevPrime P = T.primes[limb];
        u64 v = t[(size_t)poly * t_stride + j];
        u64 r = reduce64(v, P);
        if (v > half) r = sub_mod(r, reduce64(Pt.q, P), P.q);
        u[i] = r;
    }
}
void rescale_lift(const Tables &T, uint64_t *u, const uint64_t *t, int top_prime, int nlimb, int npoly,
                  size_t t_poly_stride, hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_rescale_lift, grid_for(total), dim3(256), 0, s, u, t, top_prime, T.logN, nlimb, total,
                       t_poly_stride, T);
}

__global__ void k_sub_mul(u64 *out, const u64 *c, const u64 *u, LimbConsts inv, int logN, int nlimb, size_t total,
                          size_t c_stride, LimbMap m, Tables T) {
    const size_t N = (size_t)1 << logN;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        const size_t rem = ((size_t)limb << logN) | (i & (N - 1));
        u64 q = T.primes[m.p[limb]].q;
        out[i] = mul_shoup(sub_mod(c[(size_t)poly * c_stride + rem], u[i], q), inv.v[limb], inv.sh[limb], q);
    }
}
void sub_mul(const Tables &T, uint64_t *out, const uint64_t *c, const uint64_t *u, const LimbConsts &inv, int nlimb,
             int npoly, size_t c_poly_stride, const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_sub_mul, grid_for(total), dim3(256), 0, s, out, c, u, inv, T.logN, nlimb, total,
                       c_poly_stride, m, T);
}

// ---------------------------------------------------------------------------
// Fast base conversion
// ---------------------------------------------------------------------------
// One thread per coefficient j of a polynomial: the DIN input residues are
// scaled by [Dhat_i^-1]_{q_i} (kept in registers: DIN is a template
// parameter, so the arrays are fully unrolled), then each output limb is one
// multiply-accumulate over them, reduced once.
// blockIdx.z splits the output limbs into chunks of `per` (each chunk scales
// the inputs again): more and shorter waves when a call covers few polys.
//
// SPLIT (every prime of the conversion below 2^60): residues and matrix
// entries are cut at bit 30, y = y1 2^30 + y0 and m = m1 2^30 + m0, and the
// four partial sums  sum y0 m0, sum y0 m1, sum y1 m0, sum y1 m1  are kept in
// separate 64-bit accumulators; each term is below 2^60, so up to 16 inputs
// add up without a carry, and each term is one 32 x 32 + 64-bit multiply-add.
// The sums are joined into the same 128-bit value sum y m as the plain
// 128-bit accumulation, so the reduced output is identical.
DEV void join30(u64 &hi, u64 &lo, u64 l, u64 a, u64 b, u64 h) {
    const u64 m = a + b, mc = m < a;   // a + b = mc 2^64 + m
    lo = l + (m << 30);
    hi = (m >> 34) + (mc << 30) + (lo < l);
    const u64 t = h << 60;
    lo += t;
    hi += (h >> 4) + (lo < t);
}
DEV u64 mad32(uint32_t a, uint32_t b, u64 c) { return (u64)a * b + c; }

template <int DIN, bool SPLIT>
__global__ void __launch_bounds__(256) k_bconv(u64 *__restrict__ out, const u64 *__restrict__ in,
                                               const u64 *__restrict__ mat, BconvArgs a, int logN, size_t in_stride,
                                               size_t out_stride, int per, Tables T) {
    const size_t N = (size_t)1 << logN;
    const int poly = blockIdx.y;
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int r0 = blockIdx.z * per;
    const int r1 = r0 + per < a.dout ? r0 + per : a.dout;
    u64 y[DIN];
    const u64 *src = in + poly * in_stride;
#pragma unroll
    for (int i = 0; i < DIN; ++i) {
        const u64 q = T.primes[a.pin.p[i]].q;
        y[i] = mul_shoup(src[(size_t)i * N + j], a.hinv[i], a.hinv_sh[i], q);
    }
    u64 *dst = out + poly * out_stride;
    int r = r0;
    if (SPLIT) {
        constexpr u64 kLow30 = (1ull << 30) - 1;
        uint32_t y0[DIN], y1[DIN];
#pragma unroll
        for (int i = 0; i < DIN; ++i) {
            y0[i] = (uint32_t)(y[i] & kLow30);
            y1[i] = (uint32_t)(y[i] >> 30);
        }
        for (; r + 1 < r1; r += 2) {
            const DevPrime P0 = T.primes[a.pout.p[r]], P1 = T.primes[a.pout.p[r + 1]];
            u64 l0 = 0, a0 = 0, b0 = 0, h0 = 0, l1 = 0, a1 = 0, b1 = 0, h1 = 0;
#pragma unroll
            for (int i = 0; i < DIN; ++i) {
                const u64 m = mat[(size_t)r * DIN + i], n = mat[(size_t)(r + 1) * DIN + i];
                const uint32_t m0 = (uint32_t)(m & kLow30), m1 = (uint32_t)(m >> 30);
                const uint32_t n0 = (uint32_t)(n & kLow30), n1 = (uint32_t)(n >> 30);
                l0 = mad32(y0[i], m0, l0);
                a0 = mad32(y0[i], m1, a0);
                b0 = mad32(y1[i], m0, b0);
                h0 = mad32(y1[i], m1, h0);
                l1 = mad32(y0[i], n0, l1);
                a1 = mad32(y0[i], n1, a1);
                b1 = mad32(y1[i], n0, b1);
                h1 = mad32(y1[i], n1, h1);
            }
            u64 hi0, lo0, hi1, lo1;
            join30(hi0, lo0, l0, a0, b0, h0);
            join30(hi1, lo1, l1, a1, b1, h1);
            dst[(size_t)r * N + j] = reduce128(hi0, lo0, P0);
            dst[(size_t)(r + 1) * N + j] = reduce128(hi1, lo1, P1);
        }
        if (r < r1) {
            const DevPrime P = T.primes[a.pout.p[r]];
            u64 l0 = 0, a0 = 0, b0 = 0, h0 = 0;
#pragma unroll
            for (int i = 0; i < DIN; ++i) {
                const u64 m = mat[(size_t)r * DIN + i];
                const uint32_t m0 = (uint32_t)(m & kLow30), m1 = (uint32_t)(m >> 30);
                l0 = mad32(y0[i], m0, l0);
                a0 = mad32(y0[i], m1, a0);
                b0 = mad32(y1[i], m0, b0);
                h0 = mad32(y1[i], m1, h0);
            }
            u64 hi, lo;
            join30(hi, lo, l0, a0, b0, h0);
            dst[(size_t)r * N + j] = reduce128(hi, lo, P);
        }
        return;
    }
    // two output limbs at a time: two independent 128-bit accumulation chains
    for (; r + 1 < r1; r += 2) {
        const DevPrime P0 = T.primes[a.pout.p[r]], P1 = T.primes[a.pout.p[r + 1]];
        u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
#pragma unroll
        for (int i = 0; i < DIN; ++i) {
            mac128(h0, l0, y[i], mat[(size_t)r * DIN + i]);
            mac128(h1, l1, y[i], mat[(size_t)(r + 1) * DIN + i]);
        }
        dst[(size_t)r * N + j] = reduce128(h0, l0, P0);
        dst[(size_t)(r + 1) * N + j] = reduce128(h1, l1, P1);
    }
    if (r < r1) {
        const DevPrime P = T.primes[a.pout.p[r]];
        u64 hi = 0, lo = 0;
#pragma unroll
        for (int i = 0; i < DIN; ++i) mac128(hi, lo, y[i], mat[(size_t)r * DIN + i]);
        dst[(size_t)r * N + j] = reduce128(hi, lo, P);
    }
}
template <int DIN>
static void bconv_launch(const Tables &T, uint64_t *out, const uint64_t *in, const BconvArgs &a, int npoly,
                         size_t in_poly_stride, size_t out_poly_stride, hipStream_t s) {
    const size_t N = (size_t)1 << T.logN;
    const int bx = (int)((N + 255) / 256);
    // aim at >= 2048 blocks (8 waves per SIMD) with chunks of >= 4 outputs
    int nchunk = (2048 + bx * npoly - 1) / (bx * npoly);
    const int max_chunk = (a.dout + 3) / 4;
    if (nchunk > max_chunk) nchunk = max_chunk;
    if (nchunk < 1) nchunk = 1;
    const int per = (a.dout + nchunk - 1) / nchunk;
    nchunk = (a.dout + per - 1) / per;
    dim3 grid((unsigned)bx, npoly, nchunk);
    if (a.split)
        hipLaunchKernelGGL((k_bconv<DIN, true>), grid, dim3(256), 0, s, out, in, a.mat, a, T.logN, in_poly_stride,
                           out_poly_stride, per, T);
    else
        hipLaunchKernelGGL((k_bconv<DIN, false>), grid, dim3(256), 0, s, out, in, a.mat, a, T.logN, in_poly_stride,
                           out_poly_stride, per, T);
}
void bconv(const Tables &T, uint64_t *out, const uint64_t *in, const BconvArgs &a, int npoly, size_t in_poly_stride,
           size_t out_poly_stride, hipStream_t s) {
    if (npoly <= 0 || a.dout <= 0) return;
    switch (a.din) {
#define BCONV_CASE(D) \
    case D: bconv_launch<D>(T, out, in, a, npoly, in_poly_stride, out_poly_stride, s); break;
        BCONV_CASE(1) BCONV_CASE(2) BCONV_CASE(3) BCONV_CASE(4) BCONV_CASE(5) BCONV_CASE(6) BCONV_CASE(7)
        BCONV_CASE(8) BCONV_CASE(9) BCONV_CASE(10) BCONV_CASE(11) BCONV_CASE(12) BCONV_CASE(13) BCONV_CASE(14)
        BCONV_CASE(15) BCONV_CASE(16)
#undef BCONV_CASE
        default: break;   // the host rejects digits of more than 16 primes
    }
}

// ---------------------------------------------------------------------------
// Key inner product
// ---------------------------------------------------------------------------
__global__ void k_key_inner(u64 *acc, InnerArgs a, int logN, size_t total, Tables T) {
    const size_t N = (size_t)1 << logN;
    GRID_LOOP(i, total) {
        const int e = (int)(i >> logN);
        const size_t j = i & (N - 1);
        const size_t jx = a.perm ? (size_t)a.perm[j] : j;
        const int pi = a.m.p[e];
        const DevPrime P = T.primes[pi];
        if (a.ndig <= 4) {
            // up to 4 digits: every key word of the thread loaded once, up
            // front, then per ciphertext all digits' words loaded together
            u64 k0v[4], k1v[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const bool on = d < a.ndig;
                k0v[d] = on ? a.key[(((size_t)d * 2 + 0) * a.np + pi) * N + j] : 0;
                k1v[d] = on ? a.key[(((size_t)d * 2 + 1) * a.np + pi) * N + j] : 0;
            }
            for (int b = 0; b < a.nct; ++b) {
                u64 xv[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if (d >= a.ndig) {
                        xv[d] = 0;
                    } else if (e >= a.lo[d] && e < a.hi[d]) {
                        xv[d] = a.dsrc[b * a.dsrc_stride + (size_t)e * N + jx];
                    } else {
                        const int ce = e < a.lo[d] ? e : e - (a.hi[d] - a.lo[d]);
                        xv[d] = a.ext[d][b * a.ext_stride[d] + (size_t)ce * N + jx];
                    }
                }
                u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if (d >= a.ndig) break;
                    mac128(h0, l0, xv[d], k0v[d]);
                    mac128(h1, l1, xv[d], k1v[d]);
                }
                u64 *o = acc + (size_t)b * 2 * a.ne * N;
                o[i] = reduce128(h0, l0, P);
                o[(size_t)a.ne * N + i] = reduce128(h1, l1, P);
            }
            continue;
        }
        for (int b = 0; b < a.nct; ++b) {
            u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
            for (int d = 0; d < a.ndig; ++d) {
                u64 x;
                if (e >= a.lo[d] && e < a.hi[d]) x = a.dsrc[b * a.dsrc_stride + (size_t)e * N + jx];
                else {
                    int ce = e < a.lo[d] ? e : e - (a.hi[d] - a.lo[d]);
                    x = a.ext[d][b * a.ext_stride[d] + (size_t)ce * N + jx];
                }
                const u64 *k0 = a.key + (((size_t)d * 2 + 0) * a.np + pi) * N;
                const u64 *k1 = a.key + (((size_t)d * 2 + 1) * a.np + pi) * N;
                mac128(h0, l0, x, k0[j]);
                mac128(h1, l1, x, k1[j]);
            }
            u64 *o = acc + (size_t)b * 2 * a.ne * N;
            o[i] = reduce128(h0, l0, P);
            o[(size_t)a.ne * N + i] = reduce128(h1, l1, P);
        }
    }
}
void key_inner(const Tables &T, uint64_t *acc, const InnerArgs &a, hipStream_t s) {
    size_t total = (size_t)a.ne << T.logN;
    hipLaunchKernelGGL(k_key_inner, grid_for(total), dim3(256), 0, s, acc, a, T.logN, total, T);
}

__global__ void k_key_inner_jobs(u64 *acc, InnerArgs a, KsJobs J, int logN, size_t total, Tables T) {
    const size_t N = (size_t)1 << logN;
    GRID_LOOP(i, total) {
        const int e = (int)(i >> logN);
        const size_t j = i & (N - 1);
        const int pi = a.m.p[e];
        const DevPrime P = T.primes[pi];
        // the next job's permutation word is loaded while the current job's
        // digits (read at the permuted index) are being gathered
        size_t jxn = J.perm[0] ? (size_t)J.perm[0][j] : j;
        for (int t = 0; t < J.njob; ++t) {
            const size_t jx = jxn;
            if (t + 1 < J.njob) jxn = J.perm[t + 1] ? (size_t)J.perm[t + 1][j] : j;
            const u64 *key = J.key[t];
            for (int b = 0; b < J.B; ++b) {
                const size_t ct = (size_t)(J.ct0[t] + b);
                u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
                for (int d = 0; d < a.ndig; ++d) {
                    u64 x;
                    if (e >= a.lo[d] && e < a.hi[d]) x = a.dsrc[ct * a.dsrc_stride + (size_t)e * N + jx];
                    else {
                        int ce = e < a.lo[d] ? e : e - (a.hi[d] - a.lo[d]);
                        x = a.ext[d][ct * a.ext_stride[d] + (size_t)ce * N + jx];
                    }
                    const u64 *k0 = key + (((size_t)d * 2 + 0) * a.np + pi) * N;
                    const u64 *k1 = key + (((size_t)d * 2 + 1) * a.np + pi) * N;
                    mac128(h0, l0, x, k0[j]);
                    mac128(h1, l1, x, k1[j]);
                }
                u64 *o = acc + ((size_t)t * J.B + b) * 2 * a.ne * N;
                o[i] = reduce128(h0, l0, P);
                o[(size_t)a.ne * N + i] = reduce128(h1, l1, P);
            }
        }
    }
}
void key_inner_jobs(const Tables &T, uint64_t *acc, const InnerArgs &a, const KsJobs &j, hipStream_t s) {
    size_t total = (size_t)a.ne << T.logN;
    if (!total || j.njob <= 0) return;
    hipLaunchKernelGGL(k_key_inner_jobs, grid_for(total), dim3(256), 0, s, acc, a, j, T.logN, total, T);
}

__global__ void k_key_inner_jobs_sum(u64 *acc, InnerArgs a, KsJobs J, int accumulate, int logN, size_t total,
                                     Tables T) {
    const size_t N = (size_t)1 << logN;
    GRID_LOOP(i, total) {
        const int e = (int)(i >> logN);
        const size_t j = i & (N - 1);
        const int pi = a.m.p[e];
        const DevPrime P = T.primes[pi];
        for (int b = 0; b < J.B; ++b) {
            u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;   // < 2^127 for up to 128 terms of < 2^120
            size_t jxn = J.perm[0] ? (size_t)J.perm[0][j] : j;   // one job ahead, as above
            for (int t = 0; t < J.njob; ++t) {
                const size_t jx = jxn;
                if (t + 1 < J.njob) jxn = J.perm[t + 1] ? (size_t)J.perm[t + 1][j] : j;
                const u64 *key = J.key[t];
                const size_t ct = (size_t)(J.ct0[t] + b);
                for (int d = 0; d < a.ndig; ++d) {
                    u64 x;
                    if (e >= a.lo[d] && e < a.hi[d]) x = a.dsrc[ct * a.dsrc_stride + (size_t)e * N + jx];
                    else {
                        int ce = e < a.lo[d] ? e : e - (a.hi[d] - a.lo[d]);
                        x = a.ext[d][ct * a.ext_stride[d] + (size_t)ce * N + jx];
                    }
                    const u64 *k0 = key + (((size_t)d * 2 + 0) * a.np + pi) * N;
                    const u64 *k1 = key + (((size_t)d * 2 + 1) * a.np + pi) * N;
                    mac128(h0, l0, x, k0[j]);
                    mac128(h1, l1, x, k1[j]);
                }
            }
            u64 *o = acc + (size_t)b * 2 * a.ne * N;
            u64 v0 = reduce128(h0, l0, P), v1 = reduce128(h1, l1, P);
            if (accumulate) {
                v0 = add_mod(v0, o[i], P.q);
                v1 = add_mod(v1, o[(size_t)a.ne * N + i], P.q);
            }
            o[i] = v0;
            o[(size_t)a.ne * N + i] = v1;
        }
    }
}
void key_inner_jobs_sum(const Tables &T, uint64_t *acc, const InnerArgs &a, const KsJobs &j, bool accumulate,
                        hipStream_t s) {
    size_t total = (size_t)a.ne << T.logN;
    if (!total || j.njob <= 0) return;
    hipLaunchKernelGGL(k_key_inner_jobs_sum, grid_for(total), dim3(256), 0, s, acc, a, j, (int)accumulate, T.logN,
                       total, T);
}

__global__ void k_rot_c0_sum(FinishJobs F, u64 *out, const u64 *extra, int accumulate, int logN, int nlimb, int njob,
                             size_t total, LimbMap m, Tables T) {
    const size_t N = (size_t)1 << logN;
    const size_t member = (size_t)2 * nlimb * N;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, r2, limb)   // r2 = 2 b + pp over the output batch
        const uint32_t b = r2 >> 1, pp = r2 & 1u;
        const size_t j = i & (N - 1);
        const u64 q = T.primes[m.p[limb]].q;
        u64 sum = accumulate ? out[i] : (extra ? extra[i] : 0);
        if (pp == 0)
            for (int t = 0; t < njob; ++t) {
                const size_t jx = F.perm[t] ? (size_t)F.perm[t][j] : j;
                sum = add_mod(sum, F.add[t][b * member + ((size_t)limb << logN) + jx], q);
            }
        out[i] = sum;
    }
}
// the same with 4 words per thread (N >= 1024): a block covers 1024
// consecutive words of one row (block-uniform member, poly and limb); the
// jobs go in groups of 4, each group's permutation words loaded together and
// then its 16 gathers
__global__ void __launch_bounds__(256) k_rot_c0_sum4(FinishJobs F, u64 *out, const u64 *extra, int accumulate,
                                                     int logN, int nlimb, int njob, size_t total, LimbMap m,
                                                     Tables T) {
    const size_t N = (size_t)1 << logN;
    const size_t member = (size_t)2 * nlimb * N;
    for (size_t base = (size_t)blockIdx.x * 1024; base < total; base += (size_t)gridDim.x * 1024) {
        const uint32_t row_ = (uint32_t)(base >> logN);
        const uint32_t r2 = row_ / (uint32_t)nlimb;
        const uint32_t limb = row_ - r2 * (uint32_t)nlimb;
        const uint32_t b = r2 >> 1, pp = r2 & 1u;
        const size_t j0 = (base & (N - 1)) + threadIdx.x;
        const size_t i0 = base + threadIdx.x;
        const u64 q = T.primes[m.p[limb]].q;
        u64 sum[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) sum[e] = accumulate ? out[i0 + 256 * e] : (extra ? extra[i0 + 256 * e] : 0);
        if (pp == 0) {
            const size_t rowoff = b * member + ((size_t)limb << logN);
            for (int t0 = 0; t0 < njob; t0 += 4) {
                size_t jx[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = t0 + u;
                    const int32_t *pm = t < njob ? F.perm[t] : nullptr;
#pragma unroll
                    for (int e = 0; e < 4; ++e) jx[u][e] = pm ? (size_t)pm[j0 + 256 * e] : j0 + 256 * e;
                }
                u64 w[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = t0 + u;
#pragma unroll
                    for (int e = 0; e < 4; ++e) w[u][e] = t < njob ? F.add[t][rowoff + jx[u][e]] : 0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (t0 + u >= njob) break;
#pragma unroll
                    for (int e = 0; e < 4; ++e) sum[e] = add_mod(sum[e], w[u][e], q);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) out[i0 + 256 * e] = sum[e];
    }
}
void rot_c0_sum(const Tables &T, const FinishJobs &f, uint64_t *out, const uint64_t *extra, bool accumulate,
                int nlimb, int njob, int B, const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * 2 * B) << T.logN;
    if (!total) return;
    if (T.logN >= 10) {
        hipLaunchKernelGGL(k_rot_c0_sum4, grid_for4(total), dim3(256), 0, s, f, out, extra, (int)accumulate, T.logN,
                           nlimb, njob, total, m, T);
        return;
    }
    hipLaunchKernelGGL(k_rot_c0_sum, grid_for(total), dim3(256), 0, s, f, out, extra, (int)accumulate, T.logN, nlimb,
                       njob, total, m, T);
}

__global__ void k_moddown_finish_jobs(FinishJobs F, const u64 *acc, size_t acc_stride, const u64 *z, LimbConsts pinv,
                                      int logN, int nlimb, int B, size_t total, LimbMap m, Tables T) {
    const size_t N = (size_t)1 << logN;
    const size_t member = (size_t)2 * nlimb * N;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        const uint32_t t = poly / (2u * (uint32_t)B);
        const uint32_t r2 = poly - t * 2u * (uint32_t)B;
        const uint32_t b = r2 >> 1, pp = r2 & 1u;
        const size_t j = i & (N - 1);
        const size_t rem = ((size_t)limb << logN) | j;
        const u64 q = T.primes[m.p[limb]].q;
        u64 v = mul_shoup(sub_mod(acc[(size_t)poly * acc_stride + rem], z[i], q), pinv.v[limb], pinv.sh[limb], q);
        if (pp == 0 && F.add[t]) {
            const size_t jx = F.perm[t] ? (size_t)F.perm[t][j] : j;
            v = add_mod(v, F.add[t][b * member + ((size_t)limb << logN) + jx], q);
        }
        F.out[t][b * member + (size_t)pp * nlimb * N + rem] = v;
    }
}
// the same with 4 words per thread (N >= 1024): a block covers 1024
// consecutive words of one row, so the job, member, poly, limb and their
// pointers and constants are block uniform; the accumulator, conversion and
// permutation words of all four are loaded before the dependent c0 gathers
__global__ void __launch_bounds__(256) k_moddown_finish_jobs4(FinishJobs F, const u64 *acc, size_t acc_stride,
                                                              const u64 *z, LimbConsts pinv, int logN, int nlimb,
                                                              int B, size_t total, LimbMap m, Tables T) {
    const size_t N = (size_t)1 << logN;
    const size_t member = (size_t)2 * nlimb * N;
    for (size_t base = (size_t)blockIdx.x * 1024; base < total; base += (size_t)gridDim.x * 1024) {
        const uint32_t row_ = (uint32_t)(base >> logN);
        const uint32_t poly = row_ / (uint32_t)nlimb;
        const uint32_t limb = row_ - poly * (uint32_t)nlimb;
        const uint32_t t = poly / (2u * (uint32_t)B);
        const uint32_t r2 = poly - t * 2u * (uint32_t)B;
        const uint32_t b = r2 >> 1, pp = r2 & 1u;
        const size_t j0 = (base & (N - 1)) + threadIdx.x;
        const size_t rem0 = ((size_t)limb << logN) | j0;
        const u64 q = T.primes[m.p[limb]].q;
        const u64 *ap = acc + (size_t)poly * acc_stride + rem0;
        const u64 *zp = z + base + threadIdx.x;
        const u64 *add = pp == 0 ? F.add[t] : nullptr;
        const int32_t *perm = F.perm[t];
        u64 x[4], y[4];
        size_t jx[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            x[e] = ap[256 * e];
            y[e] = zp[256 * e];
            jx[e] = (add && perm) ? (size_t)perm[j0 + 256 * e] : j0 + 256 * e;
        }
        u64 *o = F.out[t] + b * member + (size_t)pp * nlimb * N + rem0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            u64 v = mul_shoup(sub_mod(x[e], y[e], q), pinv.v[limb], pinv.sh[limb], q);
            if (add) v = add_mod(v, add[b * member + ((size_t)limb << logN) + jx[e]], q);
            o[256 * e] = v;
        }
    }
}
void moddown_finish_jobs(const Tables &T, const FinishJobs &f, const uint64_t *acc, size_t acc_poly_stride,
                         const uint64_t *z, const LimbConsts &pinv, int nlimb, int njob, int B, const LimbMap &m,
                         hipStream_t s) {
    size_t total = ((size_t)nlimb * 2 * njob * B) << T.logN;
    if (!total) return;
    if (T.logN >= 10) {
        hipLaunchKernelGGL(k_moddown_finish_jobs4, grid_for4(total), dim3(256), 0, s, f, acc, acc_poly_stride, z,
                           pinv, T.logN, nlimb, B, total, m, T);
        return;
    }
    hipLaunchKernelGGL(k_moddown_finish_jobs, grid_for(total), dim3(256), 0, s, f, acc, acc_poly_stride, z, pinv,
                       T.logN, nlimb, B, total, m, T);
}

__global__ void k_add_scaled_limb(u64 *dst, size_t dst_stride, const u64 *src, size_t src_stride, int logN,
                                  size_t total, int prime, u64 k, u64 k_sh, Tables T) {
    const u64 q = T.primes[prime].q;
    GRID_LOOP(i, total) {
        const size_t p = i >> logN, j = i & (((size_t)1 << logN) - 1);
        u64 *d = dst + p * dst_stride + j;
        *d = add_mod(*d, mul_shoup(src[p * src_stride + j], k, k_sh, q), q);
    }
}
void add_scaled_limb(const Tables &T, uint64_t *dst, size_t dst_stride, const uint64_t *src, size_t src_stride,
                     int npoly, int prime, uint64_t k, uint64_t k_sh, hipStream_t s) {
    const size_t total = (size_t)npoly << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_add_scaled_limb, grid_for(total), dim3(256), 0, s, dst, dst_stride, src, src_stride, T.logN,
                       total, prime, k, k_sh, T);
}
__global__ void k_sub_mul_add_scaled(u64 *out, const u64 *c, size_t c_stride, const u64 *z, const u64 *a,
                                     size_t a_stride, const u64 *inv, const u64 *inv_sh, const u64 *w,
                                     const u64 *w_sh, int logN, int nlimb, size_t total, LimbMap m, Tables T) {
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        const size_t rem = ((size_t)limb << logN) | (i & (((size_t)1 << logN) - 1));
        const u64 q = T.primes[m.p[limb]].q;
        const u64 r = mul_shoup(sub_mod(c[(size_t)poly * c_stride + rem], z[i], q), inv[limb], inv_sh[limb], q);
        out[i] = add_mod(r, mul_shoup(a[(size_t)poly * a_stride + rem], w[limb], w_sh[limb], q), q);
    }
}
void sub_mul_add_scaled(const Tables &T, uint64_t *out, const uint64_t *c, size_t c_stride, const uint64_t *z,
                        const uint64_t *a, size_t a_stride, const uint64_t *inv, const uint64_t *inv_sh,
                        const uint64_t *w, const uint64_t *w_sh, int nlimb, int npoly, const LimbMap &m,
                        hipStream_t s) {
    const size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_sub_mul_add_scaled, grid_for(total), dim3(256), 0, s, out, c, c_stride, z, a, a_stride, inv,
                       inv_sh, w, w_sh, T.logN, nlimb, total, m, T);
}

__global__ void k_moddown_finish(u64 *out, const u64 *acc, size_t acc_stride, const u64 *z, const u64 *add,
                                 int add_mask, LimbConsts pinv, int logN, int nlimb, size_t total, LimbMap m,
                                 Tables T) {
    const size_t N = (size_t)1 << logN;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        const size_t rem = ((size_t)limb << logN) | (i & (N - 1));
        u64 q = T.primes[m.p[limb]].q;
        u64 v = mul_shoup(sub_mod(acc[(size_t)poly * acc_stride + rem], z[i], q), pinv.v[limb], pinv.sh[limb], q);
        if (add && ((add_mask >> (poly & 1)) & 1)) v = add_mod(v, add[i], q);
        out[i] = v;
    }
}
void moddown_finish(const Tables &T, uint64_t *out, const uint64_t *acc, size_t acc_poly_stride, const uint64_t *z,
                    const uint64_t *add, int add_mask, const LimbConsts &pinv, int nlimb, int nct, const LimbMap &m,
                    hipStream_t s) {
    size_t total = ((size_t)nlimb * 2 * nct) << T.logN;
    hipLaunchKernelGGL(k_moddown_finish, grid_for(total), dim3(256), 0, s, out, acc, acc_poly_stride, z, add, add_mask,
                       pinv, T.logN, nlimb, total, m, T);
}

__global__ void k_pt_mac(u64 *out, MacArgs a, int logN, int nlimb, size_t total, LimbMap m, Tables T) {
    const size_t N = (size_t)1 << logN;
    GRID_LOOP(i, total) {
        ROW_SPLIT(i, logN, nlimb, poly, limb)
        (void)poly;
        const size_t rem = ((size_t)limb << logN) | (i & (N - 1));
        const DevPrime P = T.primes[m.p[limb]];
        u64 h = 0, l = 0;
        for (int t = 0; t < a.nterm; ++t) mac128(h, l, a.pt[t][rem], a.x[t][i]);
        out[i] = reduce128(h, l, P);
    }
}
void pt_mac(const Tables &T, uint64_t *out, const MacArgs &a, int nlimb, int npoly, const LimbMap &m,
            hipStream_t s) {
    size_t total = ((size_t)nlimb * npoly) << T.logN;
    if (!total) return;
    hipLaunchKernelGGL(k_pt_mac, grid_for(total), dim3(256), 0, s, out, a, T.logN, nlimb, total, m, T);
}

// one thread per (member, limb, word): both polys of every baby in registers
// (NB is a template parameter so that the arrays stay in registers), then one
// accumulation per giant; the next giant's plaintext words are loaded while
// the current giant's products are summed
template <int NB>
__global__ void __launch_bounds__(256) k_pt_mac_giants(u64 *out, size_t gstride, GiantArgs a, int logN, int nlimb,
                                                       size_t total, LimbMap m, Tables T) {
    const size_t N = (size_t)1 << logN;
    const size_t per = (size_t)nlimb << logN;   // words of one poly
    GRID_LOOP(i, total) {
        const uint32_t row = (uint32_t)(i >> logN);
        const uint32_t mb = row / (uint32_t)nlimb;
        const uint32_t e = row - mb * (uint32_t)nlimb;
        const size_t rem = ((size_t)e << logN) | (i & (N - 1));
        const size_t base = (size_t)mb * 2 * per + rem;
        const DevPrime P = T.primes[m.p[e]];
        u64 x0[NB], x1[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            x0[b] = a.x[b][base];
            x1[b] = a.x[b][base + per];
        }
        u64 wn[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) wn[b] = a.pt[0][b] ? a.pt[0][b][rem] : 0;
        for (int k = 0; k < a.ng; ++k) {
            u64 w[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) w[b] = wn[b];
            if (k + 1 < a.ng) {
#pragma unroll
                for (int b = 0; b < NB; ++b) wn[b] = a.pt[k + 1][b] ? a.pt[k + 1][b][rem] : 0;
            }
            u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (a.pt[k][b]) {
                    mac128(h0, l0, w[b], x0[b]);
                    mac128(h1, l1, w[b], x1[b]);
                }
            }
            u64 *o = out + k * gstride + base;
            o[0] = reduce128(h0, l0, P);
            o[per] = reduce128(h1, l1, P);
        }
    }
}
void pt_mac_giants(const Tables &T, uint64_t *out, size_t gstride, const GiantArgs &a, int nlimb, int B,
                   const LimbMap &m, hipStream_t s) {
    const size_t total = ((size_t)nlimb * B) << T.logN;
    if (!total || a.ng <= 0) return;
    switch (a.nb) {
#define GIANT_CASE(D)                                                                                            \
    case D:                                                                                                      \
        hipLaunchKernelGGL(k_pt_mac_giants<D>, grid_for(total), dim3(256), 0, s, out, gstride, a, T.logN, nlimb, \
                           total, m, T);                                                                         \
        break;
        GIANT_CASE(1) GIANT_CASE(2) GIANT_CASE(3) GIANT_CASE(4) GIANT_CASE(5) GIANT_CASE(6) GIANT_CASE(7)
        GIANT_CASE(8) GIANT_CASE(9) GIANT_CASE(10) GIANT_CASE(11) GIANT_CASE(12) GIANT_CASE(13) GIANT_CASE(14)
        GIANT_CASE(15) GIANT_CASE(16)
#undef GIANT_CASE
        default: break;   // the host checks nb <= kMaxBaby
    }
}

// UNI (N >= 64): the 64 words of a wave lie in one row (waves start at
// multiples of 64), so the row, its prime and the terms' residues are wave
// uniform and are computed once per wave on the scalar unit
template <bool UNI>
__global__ void k_lincomb(u64 *out, CombArgs a, int logN, int nlimb, size_t total, LimbMap m, Tables T) {
    const size_t N = (size_t)1 << logN;
    GRID_LOOP(i, total) {
        uint32_t row_ = (uint32_t)(i >> logN);
        if (UNI) row_ = __builtin_amdgcn_readfirstlane(row_);
        const uint32_t poly = row_ / (uint32_t)nlimb;
        const uint32_t limb = row_ - poly * (uint32_t)nlimb;
        const uint32_t b = poly >> 1, pp = poly & 1u;
        const size_t j = i & (N - 1);
        const DevPrime P = T.primes[m.p[limb]];
        u64 h = 0, l = 0;
        // terms in groups of 8: the group's loads are all issued before its
        // multiply-accumulates, so a wave keeps several loads in flight
        for (int t0 = 0; t0 < a.nterm; t0 += 8) {
            u64 xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u;
                xv[u] = t < a.nterm
                            ? a.x[t][b * a.member_stride[t] + pp * a.poly_stride[t] + ((size_t)limb << logN) + j]
                            : 0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u;
                if (t >= a.nterm) break;
                const int64_t k = a.k[t];
                u64 kv = reduce64(k < 0 ? (u64)(-(k + 1)) + 1 : (u64)k, P);
                if (k < 0 && kv) kv = P.q - kv;
                mac128(h, l, xv[u], kv);
            }
        }
        out[i] = reduce128(h, l, P);
    }
}
// A block covers 512 consecutive words of one row (N >= 512), 2 per thread,
// so the block computes the row's residues of every k[s][t] once, in LDS.
// The terms' words are loaded before that (they do not depend on it), so
// their latency overlaps the residue computation and its barriers.  The loop
// runs over block starts: every thread of a block takes the same number of
// iterations and reaches every barrier.
__global__ void __launch_bounds__(256) k_lincomb_multi(u64 *out, CombMultiArgs a, int logN, int nlimb, size_t total,
                                                       LimbMap m, Tables T) {
    __shared__ u64 kres[kMaxSum * kMaxComb];
    const size_t N = (size_t)1 << logN;
    const int nt = a.c.nterm, nk = a.nsum * nt;
    for (size_t base = (size_t)blockIdx.x * 512; base < total; base += (size_t)gridDim.x * 512) {
        const uint32_t row_ = (uint32_t)(base >> logN);
        const uint32_t poly = row_ / (uint32_t)nlimb;
        const uint32_t limb = row_ - poly * (uint32_t)nlimb;
        const uint32_t b = poly >> 1, pp = poly & 1u;
        const size_t j0 = (base & (N - 1)) + threadIdx.x;
        u64 xv[kMaxComb][2];
#pragma unroll
        for (int t = 0; t < kMaxComb; ++t) {
            const u64 *px = t < nt ? a.c.x[t] + b * a.c.member_stride[t] + pp * a.c.poly_stride[t] +
                                         ((size_t)limb << logN) + j0
                                   : nullptr;
            xv[t][0] = px ? px[0] : 0;
            xv[t][1] = px ? px[256] : 0;
        }
        const DevPrime P = T.primes[m.p[limb]];
        __syncthreads();   // the previous row's residues are no longer read
        if ((int)threadIdx.x < nk) {
            const int sidx = threadIdx.x / nt, t = threadIdx.x - sidx * nt;
            const int64_t k = a.k[sidx][t];
            u64 kv = reduce64(k < 0 ? (u64)(-(k + 1)) + 1 : (u64)k, P);
            if (k < 0 && kv) kv = P.q - kv;
            kres[threadIdx.x] = kv;
        }
        __syncthreads();
        const size_t i0 = base + threadIdx.x;
        for (int sidx = 0; sidx < a.nsum; ++sidx) {
            u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
#pragma unroll
            for (int t = 0; t < kMaxComb; ++t)
                if (t < nt) {
                    const u64 kv = kres[sidx * nt + t];
                    mac128(h0, l0, xv[t][0], kv);
                    mac128(h1, l1, xv[t][1], kv);
                }
            out[sidx * a.out_stride + i0] = reduce128(h0, l0, P);
            out[sidx * a.out_stride + i0 + 256] = reduce128(h1, l1, P);
        }
    }
}
void lincomb_multi(const Tables &T, uint64_t *out, const CombMultiArgs &a, int nlimb, int B, const LimbMap &m,
                   hipStream_t s) {
    const size_t total = ((size_t)nlimb * 2 * B) << T.logN;
    if (!total || a.c.nterm <= 0 || a.nsum <= 0) return;
    size_t nb = (total + 511) / 512;
    if (nb > 65535u * 8u) nb = 65535u * 8u;
    hipLaunchKernelGGL(k_lincomb_multi, dim3((unsigned)nb), dim3(256), 0, s, out, a, T.logN, nlimb, total, m, T);
}
// 4 words per thread (N >= 1024): a block covers 1024 consecutive words of
// one row (so the row, its prime and the terms' residues are block uniform);
// four terms' loads (16 words) are issued before their multiply-accumulates
__global__ void __launch_bounds__(256) k_lincomb4(u64 *out, CombArgs a, int logN, int nlimb, size_t total, LimbMap m,
                                                  Tables T) {
    const size_t N = (size_t)1 << logN;
    for (size_t base = (size_t)blockIdx.x * 1024; base < total; base += (size_t)gridDim.x * 1024) {
        const uint32_t row_ = (uint32_t)(base >> logN);
        const uint32_t poly = row_ / (uint32_t)nlimb;
        const uint32_t limb = row_ - poly * (uint32_t)nlimb;
        const uint32_t b = poly >> 1, pp = poly & 1u;
        const size_t j0 = (base & (N - 1)) + threadIdx.x;
        const DevPrime P = T.primes[m.p[limb]];
        u64 h[4] = {0, 0, 0, 0}, l[4] = {0, 0, 0, 0};
        for (int t0 = 0; t0 < a.nterm; t0 += 4) {
            u64 xv[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u;
                const u64 *px = t < a.nterm ? a.x[t] + b * a.member_stride[t] + pp * a.poly_stride[t] +
                                                  ((size_t)limb << logN) + j0
                                            : nullptr;
#pragma unroll
                for (int e = 0; e < 4; ++e) xv[u][e] = px ? px[256 * e] : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u;
                if (t >= a.nterm) break;
                const int64_t k = a.k[t];
                u64 kv = reduce64(k < 0 ? (u64)(-(k + 1)) + 1 : (u64)k, P);
                if (k < 0 && kv) kv = P.q - kv;
#pragma unroll
                for (int e = 0; e < 4; ++e) mac128(h[e], l[e], xv[u][e], kv);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) out[base + threadIdx.x + 256 * e] = reduce128(h[e], l[e], P);
    }
}
void lincomb(const Tables &T, uint64_t *out, const CombArgs &a, int nlimb, int B, const LimbMap &m, hipStream_t s) {
    size_t total = ((size_t)nlimb * 2 * B) << T.logN;
    if (!total || a.nterm <= 0) return;
    if (T.logN >= 10)
        hipLaunchKernelGGL(k_lincomb4, grid_for4(total), dim3(256), 0, s, out, a, T.logN, nlimb, total, m, T);
    else if (T.logN >= 6)
        hipLaunchKernelGGL(k_lincomb<true>, grid_for(total), dim3(256), 0, s, out, a, T.logN, nlimb, total, m, T);
    else
        hipLaunchKernelGGL(k_lincomb<false>, grid_for(total), dim3(256), 0, s, out, a, T.logN, nlimb, total, m, T);
}

__global__ void k_decrypt(u64 *mo, const u64 *c0, const u64 *c1, const u64 *sk, int logN, size_t total, LimbMap m,
                          Tables T) {
    GRID_LOOP(i, total) {
        const DevPrime P = T.primes[m.p[i >> logN]];
        mo[i] = add_mod(c0[i], mul_mod(c1[i], sk[i], P), P.q);
    }
}
void decrypt_combine(const Tables &T, uint64_t *mo, const uint64_t *c0, const uint64_t *c1, const uint64_t *sk,
                     int nlimb, const LimbMap &m_, hipStream_t s) {
    size_t total = (size_t)nlimb << T.logN;
    hipLaunchKernelGGL(k_decrypt, grid_for(total), dim3(256), 0, s, mo, c0, c1, sk, T.logN, total, m_, T);
}

// ---------------------------------------------------------------------------
// Butterfly-rate probe (a measurement aid for the choice of word size, not a
// step of the method).  Each thread holds 8 residues and applies `rounds`
// rounds of an 8-point forward transform (3 stages of 4 Cooley-Tukey
// butterflies U + w V, U - w V, distances 4, 2, 1) in registers, with no
// memory traffic in between, in one of three word forms, each lazily reduced
// as the transforms reduce it:
//   form 0: 64-bit words, q < 2^61: Shoup product from 32-bit multiplies,
//           U brought into [0, 4q) first when q >= 2^57, otherwise every
//           value reduced once per 5 rounds (15 stages; a 16-stage transform
//           reduces once) (the integer path);
//   form 1: binary64 residues, q < 2^42: the error-free product with a
//           rounded quotient, re-centred every 2 rounds (6 stages; a pass
//           of 8 stages is re-centred once) (the binary64 path);
//   form 2: 32-bit words, q < 2^30: Shoup product with a 32-bit quotient,
//           U brought into [0, 2q) first (no transform here uses it).
// ---------------------------------------------------------------------------
template <int FORM, int H, class T, class F>
__device__ __forceinline__ void probe_stage(T *v, F bfly) {
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if (!(m & H)) bfly(v[m], v[m + H]);
}
template <int FORM>
__global__ void __launch_bounds__(256) k_butterfly_rate(u64 *io, int rounds, u64 q, u64 w, u64 wsh, u64 inv64,
                                                       double wd, double wq, double qinv) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (FORM == 0) {
        u64 v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = (io[t] + 977 * m) % q;
        const u64 q4 = 4 * q;
        const bool small = q < kSmallPrime;
        auto bf = [&](u64 &a, u64 &b) {
            const u64 U = small ? a : (a >= q4 ? a - q4 : a);
            const u64 V = mul_shoup_lazy4(b, w, wsh, q);
            a = U + V;
            b = U - V + q4;
        };
        for (int r = 0; r < rounds; ++r) {
            probe_stage<0, 4>(v, bf);
            probe_stage<0, 2>(v, bf);
            probe_stage<0, 1>(v, bf);
            if (small && r % 5 == 4) {
#pragma unroll
                for (int m = 0; m < 8; ++m) v[m] = reduce_any(v[m], inv64, q);
            }
        }
        u64 acc = 0;
#pragma unroll
        for (int m = 0; m < 8; ++m) acc ^= v[m];
        io[t] = acc;
    } else if (FORM == 1) {
        double v[8];
        const double qd = (double)q;
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = (double)((io[t] + 977 * m) % q);
        auto bf = [&](double &a, double &b) {
            const double U = a;
            const double rr = fp_mulmod(b, wd, wq, qd);
            a = U + rr;
            b = U - rr;
        };
        for (int r = 0; r < rounds; ++r) {
            probe_stage<1, 4>(v, bf);
            probe_stage<1, 2>(v, bf);
            probe_stage<1, 1>(v, bf);
            if (r & 1) {
#pragma unroll
                for (int m = 0; m < 8; ++m) v[m] = fp_centre(v[m], qd, qinv);
            }
        }
        u64 acc = 0;
#pragma unroll
        for (int m = 0; m < 8; ++m) acc ^= fp_canon(v[m], qd, qinv);
        io[t] = acc;
    } else {
        uint32_t v[8];
        const uint32_t q32 = (uint32_t)q, w32 = (uint32_t)w, ws32 = (uint32_t)wsh, q2 = 2 * q32;
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = (uint32_t)((io[t] + 977 * m) % q);
        auto bf = [&](uint32_t &a, uint32_t &b) {
            const uint32_t U = a >= q2 ? a - q2 : a;
            const uint32_t V = b * w32 - __umulhi(b, ws32) * q32;   // [0, 2q)
            a = U + V;
            b = U - V + q2;
        };
        for (int r = 0; r < rounds; ++r) {
            probe_stage<2, 4>(v, bf);
            probe_stage<2, 2>(v, bf);
            probe_stage<2, 1>(v, bf);
        }
        u64 acc = 0;
#pragma unroll
        for (int m = 0; m < 8; ++m) acc ^= v[m];
        io[t] = acc;
    }
}
void butterfly_rate(int form, u64 *io, size_t threads, int rounds, u64 q, u64 w, u64 wsh, u64 inv64, double wd,
                    double wq, double qinv, hipStream_t s) {
    const dim3 grid((unsigned)(threads / 256));
    if (form == 0)
        hipLaunchKernelGGL(k_butterfly_rate<0>, grid, dim3(256), 0, s, io, rounds, q, w, wsh, inv64, wd, wq, qinv);
    else if (form == 1)
        hipLaunchKernelGGL(k_butterfly_rate<1>, grid, dim3(256), 0, s, io, rounds, q, w, wsh, inv64, wd, wq, qinv);
    else
        hipLaunchKernelGGL(k_butterfly_rate<2>, grid, dim3(256), 0, s, io, rounds, q, w, wsh, inv64, wd, wq, qinv);
}

}  // namespace gpu
