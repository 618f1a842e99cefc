// ckks_lib.hip -- host orchestration of the RNS-CKKS hot path and the C-ABI
// declared in include/ckks.h.
//
// Every homomorphic operation is a short sequence of kernel launches
// (kernels.hip) on the context's stream; the host only chooses constants,
// levels and scales.  Scale bookkeeping is binary64 with each formula
// evaluated in the order written next to it, so that the integer constants it
// decides (rint(value * s_c)) are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ckks.h"
#include "gpu.h"
#include "host_math.h"

using gpu::LimbConsts;
using gpu::LimbMap;
typedef uint64_t u64;
typedef unsigned __int128 u128;

namespace {

struct Error {
    ckks_status st;
    std::string msg;
};
[[noreturn]] void fail(ckks_status st, const std::string &m) { throw Error{st, m}; }
void hipchk(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(CKKS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Device memory pool over an optional caller arena (bump allocation) or
// hipMalloc.  Requests are rounded up to size classes (eight per octave above
// 1 MiB, so at most 12.5% is wasted) and served best-fit from the cached free
// blocks, taking any block of up to twice the class: batches of different
// sizes reuse each other's blocks instead of allocating afresh.  All users are
// ordered on one stream, so a block freed after its last kernel was queued can
// be handed to the next allocation immediately.
// ---------------------------------------------------------------------------
class Pool {
public:
    Pool(void *arena, size_t bytes) : base_((char *)arena), cap_(bytes), used_(0) {}
    ~Pool() {
        if (!base_)
            for (auto &kv : size_) (void)hipFree(kv.first);
    }
    static size_t size_class(size_t b) {
        b = (b + 255) & ~(size_t)255;
        if (b <= ((size_t)1 << 20)) return b;
        const int e = 63 - __builtin_clzll(b);
        const size_t step = (size_t)1 << (e - 3);
        return (b + step - 1) & ~(step - 1);
    }
    void *get(size_t bytes) {
        const size_t cls = size_class(bytes);
        auto it = free_.lower_bound(cls);
        if (it != free_.end() && it->first <= 2 * cls) {
            void *p = it->second.back();
            it->second.pop_back();
            cached_ -= it->first;
            note_use(it->first);
            if (it->second.empty()) free_.erase(it);
            if (capturing_) captured_.insert(p);
            return p;
        }
        void *p = nullptr;
        if (base_) {
            if (used_ + cls > cap_) fail(CKKS_E_OOM, "arena exhausted");
            p = base_ + used_;
            used_ += cls;
        } else if (hipMalloc(&p, cls) != hipSuccess) {
            // give the cached blocks back to the device and try once more
            (void)hipGetLastError();
            trim();
            if (hipMalloc(&p, cls) != hipSuccess) {
                (void)hipGetLastError();
                fail(CKKS_E_OOM, "hipMalloc failed");
            }
        }
        size_[p] = cls;
        held_ += cls;
        note_use(cls);
        if (capturing_) captured_.insert(p);
        return p;
    }
    // memory accounting (host side: a block is in use from get to put; work
    // queued on the stream keeps using it in stream order after put)
    size_t cached() const { return cached_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    void reset_peak() { peak_ = in_use_; }
    size_t arena_left() const { return base_ ? cap_ - used_ : 0; }
    // HIP graph capture: every block handed out while capturing is recorded;
    // at the end those blocks belong to the graph (its nodes address them on
    // every replay) and are not handed out again until release_graph.
    void begin_capture() {
        capturing_ = true;
        captured_.clear();
    }
    std::vector<void *> end_capture() {
        capturing_ = false;
        std::vector<void *> own(captured_.begin(), captured_.end());
        for (void *p : own) {
            graph_owned_.insert(p);
            const size_t sz = size_.at(p);
            auto it = free_.find(sz);
            if (it == free_.end()) continue;
            auto &v = it->second;
            auto f = std::find(v.begin(), v.end(), p);
            if (f == v.end()) continue;
            v.erase(f);
            cached_ -= sz;
            note_use(sz);   // held by the graph from now on
            if (v.empty()) free_.erase(it);
        }
        captured_.clear();
        return own;
    }
    // blocks of a destroyed graph (no longer held by any buffer) back to the cache
    void release_graph(const std::vector<void *> &own) {
        for (void *p : own) {
            graph_owned_.erase(p);
            const size_t sz = size_.at(p);
            free_[sz].push_back(p);
            cached_ += sz;
            in_use_ -= sz;
        }
    }
    void put(void *p) {
        if (!p) return;
        if (graph_owned_.count(p)) return;   // the graph keeps it
        const size_t sz = size_.at(p);
        free_[sz].push_back(p);
        cached_ += sz;
        in_use_ -= sz;
        if (!base_ && cached_ > kCacheLimit) trim();
    }
    // free every cached block (blocks still queued for use by earlier work on
    // the stream are safe: hipFree waits for outstanding work on the device)
    void trim() {
        if (base_ || capturing_) return;
        for (auto &kv : free_)
            for (void *p : kv.second) {
                size_.erase(p);
                (void)hipFree(p);
                held_ -= kv.first;
            }
        free_.clear();
        cached_ = 0;
    }

private:
    // bytes of free blocks kept for reuse: a bootstrapping batch of 64 cycles
    // through tens of GB of distinct block sizes; trimming below that would
    // free and re-allocate (with device synchronisation) on every step
    static constexpr size_t kCacheLimit = (size_t)192 << 30;
    void note_use(size_t sz) {
        in_use_ += sz;
        if (in_use_ > peak_) peak_ = in_use_;
    }
    char *base_;
    size_t cap_, used_, cached_ = 0, held_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, std::vector<void *>> free_;   // block size -> free blocks
    std::map<void *, size_t> size_;                // every block -> its size
    bool capturing_ = false;
    std::set<void *> captured_, graph_owned_;
};

struct Buf {
    Pool *pool = nullptr;
    u64 *p = nullptr;
    size_t bytes = 0;
    Buf() = default;
    Buf(Pool *pl, size_t words) : pool(pl), bytes(words * 8) { p = (u64 *)pl->get(bytes); }
    ~Buf() {
        if (pool && p) pool->put(p);
    }
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    Buf(Buf &&o) noexcept : pool(o.pool), p(o.p), bytes(o.bytes) { o.p = nullptr; }
    Buf &operator=(Buf &&o) noexcept {
        if (this != &o) {
            if (pool && p) pool->put(p);
            pool = o.pool; p = o.p; bytes = o.bytes;
            o.p = nullptr;
        }
        return *this;
    }
};

}  // namespace

struct ckks_ct {
    int level;
    double scale;
    int B = 1;  // ciphertexts held (all at this level and scale)
    Buf buf;    // [B][2][level+1][N]
    // a view into another object's memory (buf not owned): keeps it alive
    std::shared_ptr<ckks_ct> keep;
};

struct SwitchKey {
    Buf k;     // [dnum][2][np][N]
};

struct ConvTable {
    Buf hinv, hinv_sh, mat;
    LimbMap pin, pout;
    int din, dout;
    int split;   // every prime of the conversion below 2^60
};

struct BtsPlan;

// Default N = 2^16 transform schedule (ckks_ntt_schedule overrides it):
// calls of at most this many limbs in total use 4 / 8 words per thread.
constexpr int kNttR4Max = 128;
constexpr int kNttR8Max = 128;
// 4-word calls of at most this many limbs put 4 sub-transforms in a workgroup
constexpr int kNttS4Max = 128;
// N = 2^16 transforms of primes below 2^kNttFpBits run their butterflies in
// binary64 (exact: the bounds are in kernels.hip); larger primes on 64-bit
// integers.  The largest value the binary64 path accepts.
constexpr int kNttFpBits = 42;

struct ckks_ctx {
    ckks_params prm;
    int logN, N, L, K, alpha, dnum, np;
    hm::ChainShape shape;         // l_after = L for a plain chain
    std::unique_ptr<BtsPlan> bts;
    std::map<int, Buf> mono;      // k -> NTT of X^k over q_0..q_L
    std::vector<u64> q;
    std::vector<double> ladder;
    hipStream_t stream;
    hipStream_t cap_stream = nullptr;   // private stream for graph capture (created on first use)
    std::unique_ptr<Pool> pool;
    gpu::Tables T;
    Buf d_primes, d_fw, d_fwsh, d_iw, d_iwsh, d_ninv, d_ninvsh;
    Buf d_fwd, d_fwqd, d_iwd, d_iwqd, d_pd;   // binary64 twiddles and prime constants
    Buf d_rsinv, d_rsinvsh;       // [L+1][L+1]: (q_l)^-1 mod q_i and Shoup quotient, for rescale from level l
    Buf d_pinv, d_pinvsh;         // [L+1]: P^-1 mod q_i and Shoup quotient (ModDown)
    Buf d_pqinv, d_pqinvsh;       // [L+1][L+1]: (P q_l)^-1 mod q_i (ModDown merged with the rescale from l)
    std::string err;
    // keys
    bool have_keys = false;
    Buf sk;                       // [np][N] NTT form
    Buf pk;                       // [2][L+1][N]
    SwitchKey relin;
    std::map<int, SwitchKey> rot;
    std::map<int, Buf> perms;     // galois -> int32[N] (stored in a u64 buffer)
    std::map<std::pair<int, int>, std::unique_ptr<ConvTable>> modup;   // (level, digit)
    std::map<int, std::unique_ptr<ConvTable>> moddown;                 // level
    std::map<int, std::unique_ptr<ConvTable>> moddown_rs;              // level: {q_l} + P -> Q_{l-1}
    hm::Cdt cdt;
    // opt-in timing of kernel families with HIP events on the context stream
    struct ProfFamily {
        std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
        double bytes = 0;
        uint64_t calls = 0;
    };
    bool prof_on = false;
    // opt-in operation trace (op name, level, batch) for the cost model
    bool trace_on = false;
    int trace_mute = 0;           // > 0 inside bootstrapping (traced as one op)
    std::string trace;
    std::map<std::string, ProfFamily> prof;
    std::vector<hipEvent_t> ev_free;
    int sum_terms = 0;            // products a 128-bit accumulator may add: T (q_max - 1)^2 < 2^127
    // Chebyshev coefficients of 1/sqrt by (degree, interval): the quad-precision
    // interpolation takes O(d^2) cosines (about 1 ms of host time at degree 31,
    // 17 ms at 127), which would otherwise precede every chain's first launch
    std::map<std::tuple<int, double, double>, std::vector<double>> cheb_cf;
    int device = 0;               // the GPU the context was created on
    u64 *scratch = nullptr;       // that GPU's scratch array (entry point that allocates nothing)
    u64 words(int level) const { return (u64)2 * (level + 1) * N; }
    ~ckks_ctx();
};

// One slot-transform stage: a group matrix applied by baby-step giant-step.
struct LtStage {
    int level = 0;        // input level
    int stride = 0, g = 0;
    double sd = 0;        // plaintext scale
    std::vector<int> giant, baby;   // per term
    std::vector<Buf> pt;            // per term: [level+1][N] NTT form
};
struct BtsPlan {
    double K = 0;
    int r = 0, deg = 0;
    std::vector<double> cf;
    LtStage cts[3], stc[3];         // application order
};

ckks_ctx::~ckks_ctx() {
    {
        for (auto &f : prof)
            for (auto &e : f.second.ev) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
        for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
    }
    bts.reset();
    mono.clear();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

namespace {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
u64 shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }
u64 mod_signed(int64_t v, u64 q) {
    if (v >= 0) return (u64)v % q;
    u64 r = ((u64)(-(v + 1)) + 1) % q;
    return r ? q - r : 0;
}
LimbMap map_q(int first, int count) {
    LimbMap m{};
    for (int i = 0; i < count; ++i) m.p[i] = (uint8_t)(first + i);
    return m;
}
LimbMap map_ext(const ckks_ctx *c, int level) {   // q_0..q_level, p_0..p_{K-1}
    LimbMap m{};
    int e = 0;
    for (int i = 0; i <= level; ++i) m.p[e++] = (uint8_t)i;
    for (int k = 0; k < c->K; ++k) m.p[e++] = (uint8_t)(c->L + 1 + k);
    return m;
}
LimbMap map_list(const std::vector<int> &pr) {
    LimbMap m{};
    for (size_t i = 0; i < pr.size(); ++i) m.p[i] = (uint8_t)pr[i];
    return m;
}
void upload(Buf &b, const void *src, size_t bytes, hipStream_t s) {
    hipchk(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s), "upload");
    hipchk(hipStreamSynchronize(s), "upload sync");
}

int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

void trace_op(ckks_ctx *c, const char *op, int level, int B) {
    if (!c->trace_on || c->trace_mute > 0) return;
    c->trace += op;
    c->trace += ' ';
    c->trace += std::to_string(level);
    c->trace += ' ';
    c->trace += std::to_string(B);
    c->trace += '\n';
}

hipEvent_t prof_event(ckks_ctx *c) {
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e;
    hipchk(hipEventCreate(&e), "event");
    return e;
}
// RAII bracket: records start/stop events around a kernel family's launches
struct ProfScope {
    ckks_ctx *c;
    const char *fam;
    double bytes;
    hipEvent_t e0 = nullptr;
    ProfScope(ckks_ctx *c_, const char *f, double b) : c(c_), fam(f), bytes(b) {
        if (c->prof_on) {
            e0 = prof_event(c);
            hipchk(hipEventRecord(e0, c->stream), "event record");
        }
    }
    ~ProfScope() {
        if (!e0) return;
        hipEvent_t e1 = prof_event(c);
        if (hipEventRecord(e1, c->stream) != hipSuccess) return;
        auto &f = c->prof[fam];
        f.ev.emplace_back(e0, e1);
        f.bytes += bytes;
        f.calls += 1;
    }
};
// NTT with the profiling bracket (algorithmic bytes: one read + one write per word)
void ntt_p(ckks_ctx *c, uint64_t *data, int nlimb, int npoly, const LimbMap &m, bool inverse) {
    ProfScope ps(c, "ntt", 16.0 * (double)nlimb * npoly * c->N);
    gpu::ntt(c->T, data, nlimb, npoly, m, inverse, c->stream);
}
void ntt_oop_p(ckks_ctx *c, uint64_t *dst, const uint64_t *src, size_t src_stride, int nlimb, int npoly,
               const LimbMap &m, bool inverse) {
    ProfScope ps(c, "ntt", 16.0 * (double)nlimb * npoly * c->N);
    gpu::ntt_oop(c->T, dst, src, src_stride, nlimb, npoly, m, inverse, c->stream);
}

// ---------------------------------------------------------------------------
// context construction
// ---------------------------------------------------------------------------
u64 prod_mod(const ckks_ctx *c, const std::vector<int> &idx, int skip, u64 m);

void build_tables(ckks_ctx *c) {
    const int N = c->N, np = c->np;
    std::vector<gpu::DevPrime> dp(np);
    std::vector<u64> fw((size_t)np * N), fwsh((size_t)np * N), iw((size_t)np * N), iwsh((size_t)np * N);
    std::vector<u64> ninv(np), ninvsh(np);
    std::vector<u64> pw(N);
    std::vector<double> fwd((size_t)np * N), fwqd((size_t)np * N), iwd((size_t)np * N), iwqd((size_t)np * N);
    std::vector<double> pd((size_t)np * 4);
    for (int i = 0; i < np; ++i) {
        const u64 q = c->q[i];
        int n = 64 - __builtin_clzll(q);
        dp[i].q = q;
        dp[i].nbits = (uint32_t)n;
        dp[i].mu = (u64)(((u128)1 << (2 * n)) / q);
        u128 mu2 = (~(u128)0) / q;
        dp[i].mu2_lo = (u64)mu2;
        dp[i].mu2_hi = (u64)(mu2 >> 64);
        const u64 psi = hm::root_2n(q, N);
        const u64 ipsi = hm::invmod(psi, q);
        for (int pass = 0; pass < 2; ++pass) {
            u64 g = pass == 0 ? psi : ipsi, acc = 1;
            for (int k = 0; k < N; ++k) { pw[k] = acc; acc = hm::mulmod(acc, g, q); }
            u64 *dst = (pass == 0 ? fw.data() : iw.data()) + (size_t)i * N;
            u64 *dsh = (pass == 0 ? fwsh.data() : iwsh.data()) + (size_t)i * N;
            for (int k = 0; k < N; ++k) {
                dst[k] = pw[bitrev(k, c->logN)];
                dsh[k] = shoup(dst[k], q);
            }
        }
        ninv[i] = hm::invmod((u64)N, q);
        ninvsh[i] = shoup(ninv[i], q);
        const double qd = (double)q;
        for (int k = 0; k < N; ++k) {
            fwd[(size_t)i * N + k] = (double)fw[(size_t)i * N + k];
            fwqd[(size_t)i * N + k] = (double)fw[(size_t)i * N + k] / qd;
            iwd[(size_t)i * N + k] = (double)iw[(size_t)i * N + k];
            iwqd[(size_t)i * N + k] = (double)iw[(size_t)i * N + k] / qd;
        }
        pd[(size_t)i * 4 + 0] = qd;
        pd[(size_t)i * 4 + 1] = 1.0 / qd;
        pd[(size_t)i * 4 + 2] = (double)ninv[i];
        pd[(size_t)i * 4 + 3] = (double)ninv[i] / qd;
    }
    Pool *P = c->pool.get();
    c->d_primes = Buf(P, (np * sizeof(gpu::DevPrime) + 7) / 8);
    c->d_fw = Buf(P, (size_t)np * N);
    c->d_fwsh = Buf(P, (size_t)np * N);
    c->d_iw = Buf(P, (size_t)np * N);
    c->d_iwsh = Buf(P, (size_t)np * N);
    c->d_ninv = Buf(P, np);
    c->d_ninvsh = Buf(P, np);
    upload(c->d_primes, dp.data(), np * sizeof(gpu::DevPrime), c->stream);
    upload(c->d_fw, fw.data(), fw.size() * 8, c->stream);
    upload(c->d_fwsh, fwsh.data(), fwsh.size() * 8, c->stream);
    upload(c->d_iw, iw.data(), iw.size() * 8, c->stream);
    upload(c->d_iwsh, iwsh.data(), iwsh.size() * 8, c->stream);
    upload(c->d_ninv, ninv.data(), np * 8, c->stream);
    upload(c->d_ninvsh, ninvsh.data(), np * 8, c->stream);
    if (c->logN == 16) {
        c->d_fwd = Buf(P, (size_t)np * N);
        c->d_fwqd = Buf(P, (size_t)np * N);
        c->d_iwd = Buf(P, (size_t)np * N);
        c->d_iwqd = Buf(P, (size_t)np * N);
        upload(c->d_fwd, fwd.data(), fwd.size() * 8, c->stream);
        upload(c->d_fwqd, fwqd.data(), fwqd.size() * 8, c->stream);
        upload(c->d_iwd, iwd.data(), iwd.size() * 8, c->stream);
        upload(c->d_iwqd, iwqd.data(), iwqd.size() * 8, c->stream);
    }
    c->d_pd = Buf(P, (size_t)np * 4);
    upload(c->d_pd, pd.data(), pd.size() * 8, c->stream);
    {
        const int L1 = c->L + 1;
        std::vector<u64> rs((size_t)L1 * L1, 0), rssh((size_t)L1 * L1, 0);
        for (int l = 1; l < L1; ++l)
            for (int i = 0; i < l; ++i) {
                rs[(size_t)l * L1 + i] = hm::invmod(c->q[l] % c->q[i], c->q[i]);
                rssh[(size_t)l * L1 + i] = shoup(rs[(size_t)l * L1 + i], c->q[i]);
            }
        std::vector<u64> pv(L1), pvsh(L1);
        std::vector<int> sp;
        for (int k = 0; k < c->K; ++k) sp.push_back(c->L + 1 + k);
        for (int i = 0; i < L1; ++i) {
            pv[i] = hm::invmod(prod_mod(c, sp, -1, c->q[i]), c->q[i]);
            pvsh[i] = shoup(pv[i], c->q[i]);
        }
        c->d_pinv = Buf(P, L1);
        c->d_pinvsh = Buf(P, L1);
        upload(c->d_pinv, pv.data(), L1 * 8, c->stream);
        upload(c->d_pinvsh, pvsh.data(), L1 * 8, c->stream);
        std::vector<u64> pq((size_t)L1 * L1, 0), pqsh((size_t)L1 * L1, 0);
        for (int l = 1; l < L1; ++l)
            for (int i = 0; i < l; ++i) {
                const u64 q = c->q[i];
                pq[(size_t)l * L1 + i] = hm::mulmod(pv[i], rs[(size_t)l * L1 + i], q);
                pqsh[(size_t)l * L1 + i] = shoup(pq[(size_t)l * L1 + i], q);
            }
        c->d_pqinv = Buf(P, pq.size());
        c->d_pqinvsh = Buf(P, pq.size());
        upload(c->d_pqinv, pq.data(), pq.size() * 8, c->stream);
        upload(c->d_pqinvsh, pqsh.data(), pqsh.size() * 8, c->stream);
        c->d_rsinv = Buf(P, rs.size());
        c->d_rsinvsh = Buf(P, rs.size());
        upload(c->d_rsinv, rs.data(), rs.size() * 8, c->stream);
        upload(c->d_rsinvsh, rssh.data(), rssh.size() * 8, c->stream);
    }
    c->T.primes = (const gpu::DevPrime *)c->d_primes.p;
    c->T.fw = c->d_fw.p;
    c->T.fw_sh = c->d_fwsh.p;
    c->T.iw = c->d_iw.p;
    c->T.iw_sh = c->d_iwsh.p;
    c->T.ninv = c->d_ninv.p;
    c->T.ninv_sh = c->d_ninvsh.p;
    c->T.fw_d = (const double *)c->d_fwd.p;
    c->T.fwq_d = (const double *)c->d_fwqd.p;
    c->T.iw_d = (const double *)c->d_iwd.p;
    c->T.iwq_d = (const double *)c->d_iwqd.p;
    c->T.pd = (const double *)c->d_pd.p;
    c->T.fp_bits = c->logN == 16 ? kNttFpBits : 0;
    c->T.logN = c->logN;
    c->T.ntt_r4_max = kNttR4Max;
    c->T.ntt_r8_max = kNttR8Max;
    c->T.ntt_s4_max = kNttS4Max;
}

// product of primes (indices idx, skipping `skip`) modulo m
u64 prod_mod(const ckks_ctx *c, const std::vector<int> &idx, int skip, u64 m) {
    u64 r = 1 % m;
    for (int i : idx)
        if (i != skip) r = hm::mulmod(r, c->q[i] % m, m);
    return r;
}

ConvTable *make_conv(ckks_ctx *c, const std::vector<int> &in, const std::vector<int> &out) {
    auto t = std::make_unique<ConvTable>();
    t->din = (int)in.size();
    t->dout = (int)out.size();
    if (t->din > 16) fail(CKKS_E_PARAM, "digit too large for base conversion");
    std::vector<u64> hinv(t->din), hinvsh(t->din), mat((size_t)t->din * t->dout);
    for (int a = 0; a < t->din; ++a) {
        const u64 qi = c->q[in[a]];
        hinv[a] = hm::invmod(prod_mod(c, in, in[a], qi), qi);
        hinvsh[a] = shoup(hinv[a], qi);
        for (int r = 0; r < t->dout; ++r) mat[(size_t)r * t->din + a] = prod_mod(c, in, in[a], c->q[out[r]]);
    }
    Pool *P = c->pool.get();
    t->hinv = Buf(P, t->din);
    t->hinv_sh = Buf(P, t->din);
    t->mat = Buf(P, mat.size());
    upload(t->hinv, hinv.data(), hinv.size() * 8, c->stream);
    upload(t->hinv_sh, hinvsh.data(), hinvsh.size() * 8, c->stream);
    upload(t->mat, mat.data(), mat.size() * 8, c->stream);
    t->pin = map_list(in);
    t->pout = map_list(out);
    t->split = 1;
    for (int i : in) t->split &= c->q[i] < (1ull << 60);
    for (int i : out) t->split &= c->q[i] < (1ull << 60);
    return t.release();
}

ConvTable *modup_table(ckks_ctx *c, int level, int digit) {
    auto key = std::make_pair(level, digit);
    auto it = c->modup.find(key);
    if (it != c->modup.end()) return it->second.get();
    const int nq = level + 1;
    const int lo = digit * c->alpha, hi = std::min(nq, lo + c->alpha);
    std::vector<int> in, out;
    for (int i = lo; i < hi; ++i) in.push_back(i);
    for (int i = 0; i < nq; ++i)
        if (i < lo || i >= hi) out.push_back(i);
    for (int k = 0; k < c->K; ++k) out.push_back(c->L + 1 + k);
    ConvTable *t = make_conv(c, in, out);
    c->modup[key].reset(t);
    return t;
}
ConvTable *moddown_table(ckks_ctx *c, int level) {
    auto it = c->moddown.find(level);
    if (it != c->moddown.end()) return it->second.get();
    std::vector<int> in, out;
    for (int k = 0; k < c->K; ++k) in.push_back(c->L + 1 + k);
    for (int i = 0; i <= level; ++i) out.push_back(i);
    ConvTable *t = make_conv(c, in, out);
    c->moddown[level].reset(t);
    return t;
}

// conversion from D = {q_l, p_0..p_{K-1}} to q_0..q_{l-1} (ModDown merged
// with the rescale from level l)
ConvTable *moddown_rs_table(ckks_ctx *c, int level) {
    auto it = c->moddown_rs.find(level);
    if (it != c->moddown_rs.end()) return it->second.get();
    std::vector<int> in{level}, out;
    for (int k = 0; k < c->K; ++k) in.push_back(c->L + 1 + k);
    for (int i = 0; i < level; ++i) out.push_back(i);
    ConvTable *t = make_conv(c, in, out);
    c->moddown_rs[level].reset(t);
    return t;
}

const int32_t *perm_for(ckks_ctx *c, int g) {
    auto it = c->perms.find(g);
    if (it != c->perms.end()) return (const int32_t *)it->second.p;
    const int N = c->N, M = 2 * N;
    std::vector<int32_t> perm(N);
    for (int j = 0; j < N; ++j) {
        long long e = 2LL * bitrev(j, c->logN) + 1;
        long long ge = (e * g) % M;
        perm[j] = bitrev((int)((ge - 1) / 2), c->logN);
    }
    Buf b(c->pool.get(), (N + 1) / 2);
    upload(b, perm.data(), N * sizeof(int32_t), c->stream);
    const int32_t *p = (const int32_t *)b.p;
    c->perms.emplace(g, std::move(b));
    return p;
}

// ---------------------------------------------------------------------------
// ciphertext helpers
// ---------------------------------------------------------------------------
typedef std::unique_ptr<ckks_ct> Ct;
constexpr uint32_t kMaxBatch = 64;   // ciphertexts per batched launch sequence

Ct ct_new(ckks_ctx *c, int level, double scale, int B = 1) {
    Ct r(new ckks_ct);
    r->level = level;
    r->scale = scale;
    r->B = B;
    r->buf = Buf(c->pool.get(), c->words(level) * B);
    return r;
}
// members [first, first + B) of a batch object as a ciphertext object of their
// own, without a copy (the view keeps the batch's memory alive)
Ct ct_view(ckks_ctx *c, const std::shared_ptr<ckks_ct> &batch, int first, int B, double scale) {
    Ct v(new ckks_ct);
    v->level = batch->level;
    v->scale = scale;
    v->B = B;
    v->buf.pool = nullptr;
    v->buf.p = batch->buf.p + c->words(batch->level) * (size_t)first;
    v->buf.bytes = c->words(batch->level) * (size_t)B * 8;
    v->keep = batch;
    return v;
}
// poly p of ciphertext b
u64 *poly(const ckks_ctx *c, const ckks_ct *ct, int p, int b = 0) {
    return ct->buf.p + ((size_t)b * 2 + p) * (ct->level + 1) * c->N;
}

// a view of a's words under another scale, owning nothing: for temporaries
// of one operation whose source outlives them (never handed to a caller)
Ct ct_borrow(const ckks_ct *a, double scale) {
    Ct v(new ckks_ct);
    v->level = a->level;
    v->scale = scale;
    v->B = a->B;
    v->buf.pool = nullptr;
    v->buf.p = a->buf.p;
    v->buf.bytes = a->buf.bytes;
    return v;
}

Ct ct_copy(ckks_ctx *c, const ckks_ct *a) {
    trace_op(c, "copy", a->level, a->B);
    Ct r = ct_new(c, a->level, a->scale, a->B);
    hipchk(hipMemcpyAsync(r->buf.p, a->buf.p, c->words(a->level) * a->B * 8, hipMemcpyDeviceToDevice, c->stream),
           "copy");
    return r;
}

bool scales_match(double a, double b) { return std::fabs(a / b - 1.0) <= 9.313225746154785e-10; }

Ct op_addsub(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, bool sub) {
    if (a->level != b->level) fail(CKKS_E_LEVEL, "level mismatch");
    if (!scales_match(a->scale, b->scale)) fail(CKKS_E_SCALE, "scale mismatch");
    if (a->B != b->B) fail(CKKS_E_PARAM, "batch size mismatch");
    trace_op(c, sub ? "sub" : "add", a->level, a->B);
    Ct r = ct_new(c, a->level, a->scale, a->B);
    gpu::add(c->T, r->buf.p, a->buf.p, b->buf.p, a->level + 1, 2 * a->B, map_q(0, a->level + 1), sub, c->stream);
    return r;
}

Ct op_mul_int(ckks_ctx *c, const ckks_ct *a, int64_t k, double new_scale) {
    trace_op(c, "mul_scalar", a->level, a->B);
    Ct r = ct_new(c, a->level, new_scale, a->B);
    LimbConsts kc{};
    for (int i = 0; i <= a->level; ++i) {
        kc.v[i] = mod_signed(k, c->q[i]);
        kc.sh[i] = shoup(kc.v[i], c->q[i]);
    }
    gpu::mul_scalar(c->T, r->buf.p, a->buf.p, kc, a->level + 1, 2 * a->B, map_q(0, a->level + 1), c->stream);
    return r;
}

Ct op_mul_const(ckks_ctx *c, const ckks_ct *a, double value, double s_c) {
    double kd = std::rint(value * s_c);
    if (!(std::fabs(kd) < 4.0e18)) fail(CKKS_E_RANGE, "constant out of range");
    return op_mul_int(c, a, (int64_t)kd, a->scale * s_c);
}

Ct op_add_const(ckks_ctx *c, const ckks_ct *a, double value) {
    double kd = std::rint(value * a->scale);
    if (!(std::fabs(kd) < 4.0e18)) fail(CKKS_E_RANGE, "constant out of range");
    const int64_t k = (int64_t)kd;
    trace_op(c, "add_const", a->level, a->B);
    Ct r = ct_new(c, a->level, a->scale, a->B);
    LimbConsts kc{};
    for (int i = 0; i <= a->level; ++i) kc.v[i] = mod_signed(k, c->q[i]);
    gpu::add_scalar(c->T, r->buf.p, a->buf.p, kc, a->level + 1, 2 * a->B, map_q(0, a->level + 1), c->stream);
    return r;
}

// k a + value at a's scale in one pass: the words of op_mul_int(a, k, scale(a))
// followed by op_add_const(value)
Ct op_mul_int_add_const(ckks_ctx *c, const ckks_ct *a, int64_t k, double value) {
    const double kd = std::rint(value * a->scale);
    if (!(std::fabs(kd) < 4.0e18)) fail(CKKS_E_RANGE, "constant out of range");
    trace_op(c, "mul_scalar", a->level, a->B);
    Ct r = ct_new(c, a->level, a->scale, a->B);
    LimbConsts kc{};
    gpu::LimbWords cc{};
    for (int i = 0; i <= a->level; ++i) {
        kc.v[i] = mod_signed(k, c->q[i]);
        kc.sh[i] = shoup(kc.v[i], c->q[i]);
        cc.v[i] = mod_signed((int64_t)kd, c->q[i]);
    }
    gpu::mul_add_scalar(c->T, r->buf.p, a->buf.p, kc, cc, a->level + 1, 2 * a->B, map_q(0, a->level + 1),
                        c->stream);
    return r;
}

Ct op_drop(ckks_ctx *c, const ckks_ct *a, int level) {
    if (level < 0 || level > a->level) fail(CKKS_E_LEVEL, "bad target level");
    trace_op(c, "drop", level, a->B);
    Ct r = ct_new(c, level, a->scale, a->B);
    const size_t row = (size_t)(level + 1) * c->N * 8, src_pitch = (size_t)(a->level + 1) * c->N * 8;
    hipchk(hipMemcpy2DAsync(r->buf.p, row, a->buf.p, src_pitch, row, 2 * (size_t)a->B, hipMemcpyDeviceToDevice,
                            c->stream),
           "drop");
    return r;
}

// rescale by q_l: c' = (c - NTT(centred lift of iNTT(c_l))) * q_l^-1
Ct op_rescale(ckks_ctx *c, const ckks_ct *a) {
    const int l = a->level;
    if (l < 1) fail(CKKS_E_LEVEL, "rescale at level 0");
    trace_op(c, "rescale", l, a->B);
    const size_t N = c->N;
    const int np2 = 2 * a->B;
    Ct r = ct_new(c, l - 1, a->scale / (double)c->q[l], a->B);
    Buf t(c->pool.get(), np2 * N);
    ntt_oop_p(c, t.p, a->buf.p + (size_t)l * N, (size_t)(l + 1) * N, 1, np2, map_q(l, 1), true);
    Buf u(c->pool.get(), np2 * (size_t)l * N);
    if (c->logN == 16) {
        // lift fused into the transform's first pass, (c - u) / q_l into its last
        const size_t L1 = (size_t)c->L + 1;
        gpu::NttLift lf{t.p, N, l};
        gpu::NttEpi ep{r->buf.p, a->buf.p, (size_t)(l + 1) * N, c->d_rsinv.p + (size_t)l * L1,
                       c->d_rsinvsh.p + (size_t)l * L1, nullptr, 0};
        ProfScope ps(c, "ntt", 16.0 * (double)l * np2 * N);
        gpu::ntt16_fwd_fused(c->T, u.p, &lf, &ep, l, np2, map_q(0, l), c->stream);
        return r;
    }
    gpu::rescale_lift(c->T, u.p, t.p, l, l, np2, N, c->stream);
    ntt_p(c, u.p, l, np2, map_q(0, l), false);
    LimbConsts inv{};
    for (int i = 0; i < l; ++i) {
        inv.v[i] = hm::invmod(c->q[l] % c->q[i], c->q[i]);
        inv.sh[i] = shoup(inv.v[i], c->q[i]);
    }
    gpu::sub_mul(c->T, r->buf.p, a->buf.p, u.p, inv, l, np2, (size_t)(l + 1) * N, map_q(0, l), c->stream);
    return r;
}

// Device temporaries of a key switch: taken from the context's pool, or
// (the entry point that allocates nothing) carved in order from a fixed
// region, with mark / release for regions whose contents are dead.
struct Carver {
    u64 *base = nullptr;
    size_t cap = 0, used = 0;   // words
    u64 *take(size_t words) {
        const size_t w = (words + 31) & ~(size_t)31;   // 256-byte aligned pieces
        if (used + w > cap) fail(CKKS_E_PARAM, "scratch array too small for this operation");
        u64 *p = base + used;
        used += w;
        return p;
    }
};
// a temporary of `words` words: pool memory, or a non-owning piece of cv
Buf temp(ckks_ctx *c, Carver *cv, size_t words) {
    if (!cv) return Buf(c->pool.get(), words);
    Buf b;
    b.p = cv->take(words);
    b.bytes = words * 8;
    return b;
}

// ModUp of nct polynomials d (level l, NTT form; ciphertext b's polynomial
// at d + b * d_stride): per digit j the base conversion of the digit's limbs
// to the other primes of Q_l and P, NTT form.  The digits' own limbs stay in
// d (read in place by the inner product).
struct ModUp {
    int l = 0, nct = 0;
    Buf ext[gpu::kMaxDigits];
    gpu::InnerArgs ia{};
};
// the conversion tables of a level must exist already (no device allocation)
void need_tables(ckks_ctx *c, int l) {
    const int beta = (l + 1 + c->alpha - 1) / c->alpha;
    for (int j = 0; j < beta; ++j)
        if (c->modup.find(std::make_pair(l, j)) == c->modup.end())
            fail(CKKS_E_PARAM, "key-switching tables of this level are not built (ckks_keygen builds them)");
    if (c->moddown.find(l) == c->moddown.end())
        fail(CKKS_E_PARAM, "key-switching tables of this level are not built (ckks_keygen builds them)");
}
void modup(ckks_ctx *c, int l, const u64 *d, size_t d_stride, int nct, ModUp &mu, Carver *cv = nullptr) {
    const size_t N = c->N;
    const int nq = l + 1, ne = nq + c->K;
    const int beta = (nq + c->alpha - 1) / c->alpha;
    mu.l = l;
    mu.nct = nct;
    Buf dc = temp(c, cv, (size_t)nct * nq * N);
    ntt_oop_p(c, dc.p, d, d_stride, nq, nct, map_q(0, nq), true);
    gpu::InnerArgs &ia = mu.ia;
    ia = gpu::InnerArgs{};
    ia.ndig = beta;
    ia.nct = nct;
    for (int j = 0; j < beta; ++j) {
        ConvTable *t = modup_table(c, l, j);
        mu.ext[j] = temp(c, cv, (size_t)nct * t->dout * N);
        gpu::BconvArgs ba{t->pin, t->pout, t->din, t->dout, t->hinv.p, t->hinv_sh.p, t->mat.p, t->split};
        const int lo = j * c->alpha;
        gpu::bconv(c->T, mu.ext[j].p, dc.p + (size_t)lo * N, ba, nct, (size_t)nq * N, (size_t)t->dout * N,
                   c->stream);
        ntt_p(c, mu.ext[j].p, t->dout, nct, t->pout, false);
        ia.lo[j] = lo;
        ia.hi[j] = lo + t->din;
        ia.ext[j] = mu.ext[j].p;
        ia.ext_stride[j] = (size_t)t->dout * N;
    }
    ia.dsrc = d;
    ia.dsrc_stride = d_stride;
    ia.np = c->np;
    ia.m = map_ext(c, l);
    ia.ne = ne;
    ia.perm = nullptr;
}
// ModDown by P of the accumulators acc ([nct][2][ne][N], NTT form over Q_l
// and P): out ([nct][2][l+1][N]) receives (acc - Conv_P(acc)) P^-1 plus
// add[b][p] for the polys p selected by add_mask.  y ([2 nct][K][N]) and z
// ([2 nct][l+1][N]) are its temporaries.
void ks_moddown(ckks_ctx *c, int l, int nct, const u64 *acc, u64 *out, const u64 *add, int add_mask, u64 *y,
                u64 *z) {
    const size_t N = c->N;
    const int nq = l + 1, ne = nq + c->K;
    ConvTable *md = moddown_table(c, l);
    const int np2 = 2 * nct;
    ntt_oop_p(c, y, acc + (size_t)nq * N, (size_t)ne * N, c->K, np2, md->pin, true);
    gpu::BconvArgs bd{md->pin, md->pout, md->din, md->dout, md->hinv.p, md->hinv_sh.p, md->mat.p, md->split};
    gpu::bconv(c->T, z, y, bd, np2, (size_t)c->K * N, (size_t)nq * N, c->stream);
    if (c->logN == 16) {
        // (acc - z) P^-1 (+ add) fused into the transform's last pass
        gpu::NttEpi ep{out, acc, (size_t)ne * N, c->d_pinv.p, c->d_pinvsh.p, add, add_mask};
        ProfScope ps(c, "ntt", 16.0 * (double)nq * np2 * N);
        gpu::ntt16_fwd_fused(c->T, z, nullptr, &ep, nq, np2, map_q(0, nq), c->stream);
        return;
    }
    ntt_p(c, z, nq, np2, map_q(0, nq), false);
    LimbConsts pinv{};
    for (int i = 0; i < nq; ++i) {
        u64 pm = 1 % c->q[i];   // P mod q_i
        for (int k = 0; k < c->K; ++k) pm = hm::mulmod(pm, c->q[c->L + 1 + k] % c->q[i], c->q[i]);
        pinv.v[i] = hm::invmod(pm, c->q[i]);
        pinv.sh[i] = shoup(pinv.v[i], c->q[i]);
    }
    gpu::moddown_finish(c->T, out, acc, (size_t)ne * N, z, add, add_mask, pinv, nq, nct, map_q(0, nq), c->stream);
}
// Inner product of the ModUp digits (read through `perm`, the NTT-domain
// index map of an automorphism, when given) with the key, ModDown by P.  out
// ([nct][2][l+1][N]) receives (o0, o1) plus add[b][p] for the polys p
// selected by add_mask.
void ks_finish(ckks_ctx *c, const ModUp &mu, const SwitchKey &key, const int32_t *perm, u64 *out, const u64 *add,
               int add_mask) {
    const size_t N = c->N;
    const int l = mu.l, nct = mu.nct, nq = l + 1, ne = nq + c->K;
    Pool *P = c->pool.get();
    gpu::InnerArgs ia = mu.ia;
    ia.key = key.k.p;
    ia.perm = perm;
    Buf acc(P, (size_t)nct * 2 * ne * N);
    gpu::key_inner(c->T, acc.p, ia, c->stream);
    Buf y(P, (size_t)2 * nct * c->K * N), z(P, (size_t)2 * nct * nq * N);
    ks_moddown(c, l, nct, acc.p, out, add, add_mask, y.p, z.p);
}

// Hybrid key switch of nct polynomials d (level l, NTT form; ciphertext b's
// polynomial at d + b * d_stride).  out ([nct][2][l+1][N]) receives
// (o0, o1) plus add[b][p] for the polys p selected by add_mask.
void keyswitch(ckks_ctx *c, int l, const u64 *d, size_t d_stride, int nct, const SwitchKey &key, u64 *out,
               const u64 *add, int add_mask) {
    const size_t N = c->N;
    const int nq = l + 1, ne = nq + c->K;
    const int beta = (nq + c->alpha - 1) / c->alpha;
    // algorithmic bytes: d (nq limbs) in, key (2 beta ne limbs) in once, result (2 nq limbs) out, per ciphertext
    ProfScope ps(c, "keyswitch", 8.0 * (double)N * ((double)nct * nq + 2.0 * beta * ne + 2.0 * nct * nq));
    ModUp mu;
    modup(c, l, d, d_stride, nct, mu);
    ks_finish(c, mu, key, nullptr, out, add, add_mask);
}

Ct op_hmult(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b) {
    if (!c->have_keys) fail(CKKS_E_NOKEY, "no keys");
    if (a->level != b->level) fail(CKKS_E_LEVEL, "level mismatch");
    if (a->B != b->B) fail(CKKS_E_PARAM, "batch size mismatch");
    const int l = a->level, nq = l + 1, B = a->B;
    trace_op(c, "hmult", l, B);
    const size_t N = c->N;
    Ct r = ct_new(c, l, a->scale * b->scale, B);
    Buf d01(c->pool.get(), (size_t)B * 2 * nq * N), d2(c->pool.get(), (size_t)B * nq * N);
    gpu::tensor(c->T, d01.p, d2.p, a->buf.p, b->buf.p, nq, B, map_q(0, nq), c->stream);
    keyswitch(c, l, d2.p, (size_t)nq * N, B, c->relin, r->buf.p, d01.p, 3);
    return r;
}

// products of several pairs of equal level and batch size as one batch object
// (ciphertext k * B + j is member j of pair k); its scale is that of pair 0
// (callers that mix scales give each member its own afterwards)
Ct op_hmult_many(ckks_ctx *c, const std::vector<const ckks_ct *> &A, const std::vector<const ckks_ct *> &Bv) {
    if (!c->have_keys) fail(CKKS_E_NOKEY, "no keys");
    const int G = (int)A.size();
    if (G < 1 || G > gpu::kMaxGather || Bv.size() != A.size()) fail(CKKS_E_PARAM, "bad product list");
    const int l = A[0]->level, nq = l + 1, B = A[0]->B;
    for (int k = 0; k < G; ++k)
        if (A[k]->level != l || Bv[k]->level != l || A[k]->B != B || Bv[k]->B != B)
            fail(CKKS_E_LEVEL, "level or batch mismatch");
    trace_op(c, "hmult", l, G * B);
    const size_t N = c->N;
    Ct r = ct_new(c, l, A[0]->scale * Bv[0]->scale, G * B);
    Buf d01(c->pool.get(), (size_t)G * B * 2 * nq * N), d2(c->pool.get(), (size_t)G * B * nq * N);
    gpu::GatherPtrs gp{};
    gp.per_src = B;
    for (int k = 0; k < G; ++k) {
        gp.a[k] = A[k]->buf.p;
        gp.b[k] = Bv[k]->buf.p;
    }
    gpu::tensor_gather(c->T, d01.p, d2.p, gp, nq, G * B, map_q(0, nq), c->stream);
    keyswitch(c, l, d2.p, (size_t)nq * N, G * B, c->relin, r->buf.p, d01.p, 3);
    return r;
}

// ModDown by P q_l of t = acc + P d over np2 polys (the rescale from level l
// merged into the key switch's ModDown): acc [np2][l+1+K][N] over Q_l and P
// (its q_l limb is overwritten with t's), d [np2][l+1][N] over Q_l, out
// [np2][l][N]: out_i = (acc_i - Conv_D(t)_i) (P q_l)^-1 + d_i q_l^-1 mod q_i,
// D = {q_l} + P, with the approximate conversion.
void moddown_rescale(ckks_ctx *c, int l, u64 *acc, const u64 *d, int np2, u64 *out) {
    const size_t N = c->N;
    const int nq = l + 1, K = c->K, ne = nq + K;
    Pool *P = c->pool.get();
    std::vector<int> pidx;
    for (int k = 0; k < K; ++k) pidx.push_back(c->L + 1 + k);
    const u64 ql = c->q[l], pm = prod_mod(c, pidx, -1, ql);
    // t on q_l: acc + (P mod q_l) d
    gpu::add_scaled_limb(c->T, acc + (size_t)l * N, (size_t)ne * N, d + (size_t)l * N, (size_t)nq * N, np2, l, pm,
                         shoup(pm, ql), c->stream);
    ConvTable *md = moddown_rs_table(c, l);
    Buf y(P, (size_t)np2 * (K + 1) * N);
    ntt_oop_p(c, y.p, acc + (size_t)l * N, (size_t)ne * N, K + 1, np2, md->pin, true);
    Buf z(P, (size_t)np2 * l * N);
    gpu::BconvArgs bd{md->pin, md->pout, md->din, md->dout, md->hinv.p, md->hinv_sh.p, md->mat.p, md->split};
    gpu::bconv(c->T, z.p, y.p, bd, np2, (size_t)(K + 1) * N, (size_t)l * N, c->stream);
    const size_t L1 = (size_t)c->L + 1;
    const u64 *inv = c->d_pqinv.p + (size_t)l * L1, *inv_sh = c->d_pqinvsh.p + (size_t)l * L1;
    const u64 *w = c->d_rsinv.p + (size_t)l * L1, *w_sh = c->d_rsinvsh.p + (size_t)l * L1;
    if (c->logN == 16) {
        gpu::NttEpi ep{out, acc, (size_t)ne * N, inv, inv_sh, d, 3, (size_t)nq * N, w, w_sh};
        ProfScope pn(c, "ntt", 16.0 * (double)l * np2 * N);
        gpu::ntt16_fwd_fused(c->T, z.p, nullptr, &ep, l, np2, map_q(0, l), c->stream);
    } else {
        ntt_p(c, z.p, l, np2, map_q(0, l), false);
        gpu::sub_mul_add_scaled(c->T, out, acc, (size_t)ne * N, z.p, d, (size_t)nq * N, inv, inv_sh, w, w_sh, l, np2,
                                map_q(0, l), c->stream);
    }
}

// Mul_C, relinearisation and rescale with the rescale merged into the key
// switch's ModDown (one division by P q_l), for several pairs of equal level
// and batch size as one batch object (ciphertext k * B + j is member j of pair
// k; its scale is that of pair 0, callers give members their own).  With the
// tensor (d0, d1, d2), acc = <ModUp(d2), relin key> over Q_l and P, t = acc +
// P (d0, d1) and D = {q_l} + P: out_i = (acc_i - Conv_D(t)_i) (P q_l)^-1 +
// d_i q_l^-1 mod q_i for i < l.
Ct op_hmult_rs_many(ckks_ctx *c, const std::vector<const ckks_ct *> &A, const std::vector<const ckks_ct *> &Bv) {
    if (!c->have_keys) fail(CKKS_E_NOKEY, "no keys");
    const int G = (int)A.size();
    if (G < 1 || G > gpu::kMaxGather || Bv.size() != A.size()) fail(CKKS_E_PARAM, "bad product list");
    const int l = A[0]->level, nq = l + 1, B = A[0]->B, K = c->K, ne = nq + K;
    if (l < 1) fail(CKKS_E_LEVEL, "no level for Mul_C");
    for (int k = 0; k < G; ++k)
        if (A[k]->level != l || Bv[k]->level != l || A[k]->B != B || Bv[k]->B != B)
            fail(CKKS_E_LEVEL, "level or batch mismatch");
    trace_op(c, "hmult", l, G * B);
    trace_op(c, "rescale", l, G * B);
    const size_t N = c->N;
    const int nct = G * B, np2 = 2 * nct;
    Pool *P = c->pool.get();
    Ct r = ct_new(c, l - 1, (A[0]->scale * Bv[0]->scale) / (double)c->q[l], nct);
    Buf d01(P, (size_t)nct * 2 * nq * N), d2(P, (size_t)nct * nq * N);
    gpu::GatherPtrs gp{};
    gp.per_src = B;
    for (int k = 0; k < G; ++k) {
        gp.a[k] = A[k]->buf.p;
        gp.b[k] = Bv[k]->buf.p;
    }
    gpu::tensor_gather(c->T, d01.p, d2.p, gp, nq, nct, map_q(0, nq), c->stream);
    const int beta = (nq + c->alpha - 1) / c->alpha;
    ProfScope ps(c, "keyswitch", 8.0 * (double)N * ((double)nct * nq + 2.0 * beta * ne + 2.0 * nct * l));
    ModUp mu;
    modup(c, l, d2.p, (size_t)nq * N, nct, mu);
    gpu::InnerArgs ia = mu.ia;
    ia.key = c->relin.k.p;
    ia.perm = nullptr;
    Buf acc(P, (size_t)np2 * ne * N);
    gpu::key_inner(c->T, acc.p, ia, c->stream);
    moddown_rescale(c, l, acc.p, d01.p, np2, r->buf.p);
    return r;
}

Ct op_automorphism(ckks_ctx *c, const ckks_ct *a, int g) {
    auto it = c->rot.find(g);
    if (it == c->rot.end()) fail(CKKS_E_NOKEY, "missing Galois key");
    const int nq = a->level + 1, B = a->B;
    trace_op(c, "rotate", a->level, B);
    const size_t N = c->N;
    const int32_t *perm = perm_for(c, g);
    Buf s(c->pool.get(), (size_t)B * 2 * nq * N);
    gpu::permute(c->T, s.p, a->buf.p, perm, nq, 2 * B, c->stream);
    Ct r = ct_new(c, a->level, a->scale, B);
    // r = (sigma(c0) + ks0, ks1): key switch sigma(c1), add sigma(c0) to poly 0 only
    keyswitch(c, a->level, s.p + (size_t)nq * N, (size_t)2 * nq * N, B, it->second, r->buf.p, s.p, 1);
    return r;
}

int galois_rot(const ckks_ctx *c, int k);

// One rotation of a batch of inputs in a job list (see ks_rot_jobs).
struct RotJob {
    const SwitchKey *key;
    const int32_t *perm;
    int ct0;          // first of the job's B inputs in the ModUp
    u64 *out;         // [B][2][l+1][N]
    const u64 *add;   // [B][2][l+1][N]: its c0 (poly 0), read through perm, is added
};
// Key switching of rotation jobs over one ModUp: inner products and ModDown
// of up to kMaxJobs jobs run as one launch sequence.
void ks_rot_jobs(ckks_ctx *c, const ModUp &mu, int B, const std::vector<RotJob> &jobs) {
    const size_t N = c->N;
    const int l = mu.l, nq = l + 1, ne = nq + c->K;
    const int beta = (nq + c->alpha - 1) / c->alpha;
    Pool *P = c->pool.get();
    ConvTable *md = moddown_table(c, l);
    LimbConsts pinv{};
    std::vector<int> pidx;
    for (int k = 0; k < c->K; ++k) pidx.push_back(c->L + 1 + k);
    for (int i = 0; i < nq; ++i) {
        pinv.v[i] = hm::invmod(prod_mod(c, pidx, -1, c->q[i]), c->q[i]);
        pinv.sh[i] = shoup(pinv.v[i], c->q[i]);
    }
    // at most 64 ciphertexts' worth of extended accumulators per launch sequence
    const size_t per = (size_t)std::max(1, std::min(gpu::kMaxJobs, 64 / std::max(1, B)));
    for (size_t j0 = 0; j0 < jobs.size(); j0 += per) {
        const int nj = (int)std::min<size_t>(per, jobs.size() - j0);
        ProfScope ps(c, "keyswitch", 8.0 * (double)N * ((double)nj * 2.0 * beta * ne + 2.0 * nj * B * nq));
        gpu::KsJobs kj{};
        gpu::FinishJobs fj{};
        kj.njob = nj;
        kj.B = B;
        for (int t = 0; t < nj; ++t) {
            const RotJob &jb = jobs[j0 + t];
            kj.ct0[t] = jb.ct0;
            kj.key[t] = jb.key->k.p;
            kj.perm[t] = jb.perm;
            fj.out[t] = jb.out;
            fj.add[t] = jb.add;
            fj.perm[t] = jb.perm;
        }
        const int np2 = 2 * nj * B;
        Buf acc(P, (size_t)np2 * ne * N);
        gpu::key_inner_jobs(c->T, acc.p, mu.ia, kj, c->stream);
        Buf y(P, (size_t)np2 * c->K * N);
        ntt_oop_p(c, y.p, acc.p + (size_t)nq * N, (size_t)ne * N, c->K, np2, md->pin, true);
        Buf z(P, (size_t)np2 * nq * N);
        gpu::BconvArgs bd{md->pin, md->pout, md->din, md->dout, md->hinv.p, md->hinv_sh.p, md->mat.p, md->split};
        gpu::bconv(c->T, z.p, y.p, bd, np2, (size_t)c->K * N, (size_t)nq * N, c->stream);
        ntt_p(c, z.p, nq, np2, map_q(0, nq), false);
        gpu::moddown_finish_jobs(c->T, fj, acc.p, (size_t)ne * N, z.p, pinv, nq, nj, B, map_q(0, nq), c->stream);
    }
}

// Rotations of one ciphertext object by several steps sharing one ModUp of
// c1 (hoisting): each applies its automorphism to the digits inside the inner
// product, then ModDown, plus the permuted c0.  Step 0 gives a copy.
std::vector<Ct> op_rotate_hoisted(ckks_ctx *c, const ckks_ct *a, const std::vector<int> &steps) {
    const int l = a->level, nq = l + 1, B = a->B;
    const size_t N = c->N;
    std::vector<Ct> outs(steps.size());
    std::vector<RotJob> jobs;
    for (size_t i = 0; i < steps.size(); ++i) {
        const int g = galois_rot(c, steps[i]);
        if (g == 1) {
            outs[i] = ct_copy(c, a);
            continue;
        }
        auto it = c->rot.find(g);
        if (it == c->rot.end()) fail(CKKS_E_NOKEY, "missing Galois key");
        trace_op(c, "rotate_hoisted", l, B);
        outs[i] = ct_new(c, l, a->scale, B);
        jobs.push_back(RotJob{&it->second, perm_for(c, g), 0, outs[i]->buf.p, a->buf.p});
    }
    if (jobs.empty()) return outs;
    ModUp mu;
    {
        ProfScope ps(c, "keyswitch", 8.0 * (double)N * B * nq);
        modup(c, l, a->buf.p + (size_t)nq * N, (size_t)2 * nq * N, B, mu);
    }
    ks_rot_jobs(c, mu, B, jobs);
    return outs;
}

int galois_rot(const ckks_ctx *c, int k) {
    const int n = c->N / 2, M = 2 * c->N;
    k %= n;
    if (k < 0) k += n;
    long long g = 1;
    for (int t = 0; t < k; ++t) g = (g * 5) % M;
    return (int)g;
}

Ct op_rotate(ckks_ctx *c, const ckks_ct *a, int k) {
    int g = galois_rot(c, k);
    if (g == 1) return ct_copy(c, a);
    return op_automorphism(c, a, g);
}

// Linear combination sum_t rint(v_t s_t) x_t over the lowest level+1 limbs of
// each x_t (one kernel: no limb-drop copies, one pass over the inputs); the
// result carries the scale of the first term, scale(x_0) s_0, and every
// term's scale(x_t) s_t must match it (as for a chain of Mul_P and Add).
Ct op_lincomb(ckks_ctx *c, const std::vector<const ckks_ct *> &xs, const std::vector<double> &v,
              const std::vector<double> &sc, int level) {
    const int B = xs[0]->B;
    const size_t N = c->N;
    const double scale = xs[0]->scale * sc[0];
    Ct r = ct_new(c, level, scale, B);
    for (size_t t0 = 0; t0 < xs.size(); t0 += gpu::kMaxComb) {
        gpu::CombArgs ca{};
        const size_t t1 = std::min(xs.size(), t0 + gpu::kMaxComb);
        if (t0 > 0) {   // carry the partial sum as a term with constant 1
            ca.x[0] = r->buf.p;
            ca.member_stride[0] = (size_t)2 * (level + 1) * N;
            ca.poly_stride[0] = (size_t)(level + 1) * N;
            ca.k[0] = 1;
            ca.nterm = 1;
        }
        for (size_t t = t0; t < t1; ++t) {
            const ckks_ct *x = xs[t];
            if (x->level < level || x->B != B) fail(CKKS_E_LEVEL, "bad term for the linear combination");
            if (t > 0 && !scales_match(scale, x->scale * sc[t])) fail(CKKS_E_SCALE, "scale mismatch");
            const double kd = std::rint(v[t] * sc[t]);
            if (!(std::fabs(kd) < 4.0e18)) fail(CKKS_E_RANGE, "constant out of range");
            // one launch per chunk: its first term opens it, every further term adds one read
            trace_op(c, t == t0 ? "lincomb" : "lincomb_term", level, B);
            const int n = ca.nterm++;
            ca.x[n] = x->buf.p;
            ca.member_stride[n] = (size_t)2 * (x->level + 1) * N;
            ca.poly_stride[n] = (size_t)(x->level + 1) * N;
            ca.k[n] = (int64_t)kd;
        }
        gpu::lincomb(c->T, r->buf.p, ca, level + 1, B, map_q(0, level + 1), c->stream);
    }
    return r;
}

Ct op_level_to(ckks_ctx *c, const ckks_ct *a, int target) {
    if (target == a->level) return ct_copy(c, a);
    if (target > a->level || target < 0) fail(CKKS_E_LEVEL, "bad target level");
    double sc = (c->ladder[target] * (double)c->q[target + 1]) / a->scale;
    Ct m = op_lincomb(c, {a}, {1.0}, {sc}, target + 1);
    return op_rescale(c, m.get());
}

Ct op_mul_const_down(ckks_ctx *c, const ckks_ct *a, double value) {
    const int l = a->level;
    if (l < 1) fail(CKKS_E_LEVEL, "no level for Mul_P");
    double sc = (c->ladder[l - 1] * (double)c->q[l]) / a->scale;
    Ct m = op_mul_const(c, a, value, sc);
    return op_rescale(c, m.get());
}

// Mul_C, relinearise, rescale (the rescale merged into the ModDown)
Ct mult_rs(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b) {
    if (a->level != b->level) fail(CKKS_E_LEVEL, "level mismatch");
    if (a->B != b->B) fail(CKKS_E_PARAM, "batch size mismatch");
    return op_hmult_rs_many(c, {a}, {b});
}
Ct mult_aligned(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b) {
    int l = std::min(a->level, b->level);
    if (l < 1) fail(CKKS_E_LEVEL, "no level for Mul_C");
    Ct x = op_level_to(c, a, l), y = op_level_to(c, b, l);
    return mult_rs(c, x.get(), y.get());
}
// Products a_i * b_i, each pair aligned to the lower of its two levels (as
// mult_aligned), then multiplied and rescaled; pairs that land on the same
// level share one launch sequence (their operands copied into one batch
// object).  Words and scales of every result are exactly those of
// mult_aligned(a_i, b_i): the kernels do not read the scale, and each result
// gets (scale(a_i) scale(b_i)) / q_l as op_hmult and op_rescale compute it.
constexpr int kMaxWaveBatch = 4;   // ciphertexts per operand above which products are not regrouped
std::vector<Ct> mult_aligned_many(ckks_ctx *c, const std::vector<std::pair<const ckks_ct *, const ckks_ct *>> &pairs) {
    const size_t n = pairs.size();
    std::vector<Ct> out(n), own_a(n), own_b(n);
    std::vector<const ckks_ct *> A(n), Bc(n);
    std::vector<int> lv(n);
    for (size_t i = 0; i < n; ++i) {
        const ckks_ct *a = pairs[i].first, *b = pairs[i].second;
        const int l = std::min(a->level, b->level);
        if (l < 1) fail(CKKS_E_LEVEL, "no level for Mul_C");
        if (a->B != b->B || a->B != pairs[0].first->B) fail(CKKS_E_PARAM, "batch size mismatch");
        lv[i] = l;
        if (a->level != l) own_a[i] = op_level_to(c, a, l);
        if (b == a) own_b[i] = Ct();
        else if (b->level != l) own_b[i] = op_level_to(c, b, l);
        A[i] = own_a[i] ? own_a[i].get() : a;
        Bc[i] = b == a ? A[i] : (own_b[i] ? own_b[i].get() : b);
    }
    std::vector<char> done(n, 0);
    for (size_t i0 = 0; i0 < n; ++i0) {
        if (done[i0]) continue;
        std::vector<size_t> grp;
        for (size_t i = i0; i < n; ++i)
            if (!done[i] && lv[i] == lv[i0]) grp.push_back(i), done[i] = 1;
        const int l = lv[i0];
        if (grp.size() == 1 || A[i0]->B > kMaxWaveBatch || grp.size() > (size_t)gpu::kMaxGather) {
            // a large batch fills the GPU by itself: the copies would cost more than they save
            for (size_t i : grp) out[i] = mult_rs(c, A[i], Bc[i]);
            continue;
        }
        const int B = A[i0]->B, G = (int)grp.size();
        std::vector<const ckks_ct *> ga, gb;
        for (size_t i : grp) {
            ga.push_back(A[i]);
            gb.push_back(Bc[i]);
        }
        Ct r = op_hmult_rs_many(c, ga, gb);   // operands read in place (gathered)
        std::shared_ptr<ckks_ct> rs(r.release());
        for (int k = 0; k < G; ++k) {   // members as views of the batch, each with its own scale
            const size_t i = grp[k];
            out[i] = ct_view(c, rs, k * B, B, (A[i]->scale * Bc[i]->scale) / (double)c->q[l]);
        }
    }
    return out;
}

Ct addsub_aligned(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, bool sub) {
    int l = std::min(a->level, b->level);
    Ct x = op_level_to(c, a, l), y = op_level_to(c, b, l);
    return op_addsub(c, x.get(), y.get(), sub);
}

// ---------------------------------------------------------------------------
// Chebyshev evaluation (baby-step / giant-step), Newton, CryptoInvSqrt
// ---------------------------------------------------------------------------
struct PowerBasis {
    ckks_ctx *c;
    std::vector<Ct> T;
    ckks_ct *get(int i) {
        if (!T[i]) T[i] = make(i);
        return T[i].get();
    }
    Ct make(int i) {
        if (i % 2 == 0) {   // T_2k = 2 T_k^2 - 1
            ckks_ct *h = get(i / 2);
            Ct sq = mult_rs(c, h, h);
            return finish(i, std::move(sq));
        }
        // T_2k+1 = 2 T_k+1 T_k - T_1
        ckks_ct *hi = get((i + 1) / 2);
        ckks_ct *lo = get((i - 1) / 2);
        Ct p = mult_aligned(c, hi, lo);
        return finish(i, std::move(p));
    }
    // T_i from its product: 2 p - 1 (even i) or 2 p - T_1 (odd i)
    Ct finish(int i, Ct p) {
        if (i % 2 == 0) return op_mul_int_add_const(c, p.get(), 2, -1.0);
        // 2 p - T_1 as one linear combination, T_1 first brought to p's level
        // (and scale) when it sits higher
        Ct t1;
        const ckks_ct *u = T[1].get();
        if (u->level < p->level) {
            Ct two = op_mul_int(c, p.get(), 2, p->scale);
            return addsub_aligned(c, two.get(), u, true);
        }
        if (u->level > p->level) {
            t1 = op_level_to(c, u, p->level);
            u = t1.get();
        }
        return op_lincomb(c, {p.get(), u}, {2.0, -1.0}, {1.0, 1.0}, p->level);
    }
    // every T_i of `want` (and what they need), wave by wave: the products of
    // one wave whose operands are ready share launch sequences
    void ensure(const std::vector<int> &want) {
        std::vector<int> need;
        std::function<void(int)> add = [&](int i) {
            if (i <= 1 || T[i] || std::find(need.begin(), need.end(), i) != need.end()) return;
            need.push_back(i);
            if (i % 2 == 0) add(i / 2);
            else { add((i + 1) / 2); add((i - 1) / 2); }
        };
        for (int i : want) add(i);
        std::sort(need.begin(), need.end());
        while (!need.empty()) {
            std::vector<int> ready;
            std::vector<std::pair<const ckks_ct *, const ckks_ct *>> pairs;
            for (int i : need) {
                const int a = i % 2 == 0 ? i / 2 : (i + 1) / 2, b = i % 2 == 0 ? i / 2 : (i - 1) / 2;
                if (T[a] && T[b]) {
                    ready.push_back(i);
                    pairs.emplace_back(T[a].get(), T[b].get());
                }
            }
            if (ready.empty()) fail(CKKS_E_PARAM, "power basis: unresolved dependency");
            std::vector<Ct> P = mult_aligned_many(c, pairs);
            for (size_t k = 0; k < ready.size(); ++k) T[ready[k]] = finish(ready[k], std::move(P[k]));
            std::vector<int> rest;
            for (int i : need)
                if (!T[i]) rest.push_back(i);
            need.swap(rest);
        }
    }
};

Ct baby_sum(ckks_ctx *c, PowerBasis &pb, const std::vector<double> &cf) {
    const int deg = (int)cf.size() - 1;
    std::vector<int> terms;
    for (int i = 1; i <= deg; ++i)
        if (cf[i] != 0.0) terms.push_back(i);
    const bool none = terms.empty();
    if (none) terms.push_back(1);
    int lmin = 1 << 30;
    for (int i : terms) lmin = std::min(lmin, pb.T[i]->level);
    if (lmin < 1) fail(CKKS_E_LEVEL, "no level for the baby-step sum");
    std::vector<const ckks_ct *> xs;
    std::vector<double> v, sc;
    for (int i : terms) {
        const ckks_ct *Ti = pb.T[i].get();
        xs.push_back(Ti);
        v.push_back(none ? 0.0 : cf[i]);
        sc.push_back((c->ladder[lmin - 1] * (double)c->q[lmin]) / Ti->scale);
    }
    Ct acc = op_lincomb(c, xs, v, sc, lmin);
    Ct r = op_rescale(c, acc.get());
    return op_add_const(c, r.get(), cf[0]);
}

// The baby-step sums of several leaves at once, when they combine the same
// basis elements (every leaf of one evaluation does, unless a coefficient is
// exactly 0): one pass reads each T_i once for every leaf, the leaves' sums
// are rescaled as one batch, then each gets its constant term.  Every word
// equals baby_sum's for the leaf alone.  Returns false where it does not apply.
bool baby_sums_together(ckks_ctx *c, PowerBasis &pb, const std::vector<std::vector<double>> &cfs,
                        std::vector<Ct> &out) {
    const size_t n = cfs.size();
    if (n < 2 || n > (size_t)gpu::kMaxSum || c->logN < 9) return false;
    std::vector<int> terms;
    for (size_t t = 0; t < n; ++t) {
        std::vector<int> tt;
        for (int i = 1; i < (int)cfs[t].size(); ++i)
            if (cfs[t][i] != 0.0) tt.push_back(i);
        if (tt.empty() || (t > 0 && tt != terms)) return false;
        terms = tt;
    }
    if (terms.size() > (size_t)gpu::kMaxComb) return false;
    int lmin = 1 << 30;
    for (int i : terms) lmin = std::min(lmin, pb.T[i]->level);
    if (lmin < 1) fail(CKKS_E_LEVEL, "no level for the baby-step sum");
    const int B = pb.T[terms[0]]->B;
    const size_t N = c->N;
    const double scale = pb.T[terms[0]]->scale * ((c->ladder[lmin - 1] * (double)c->q[lmin]) / pb.T[terms[0]]->scale);
    gpu::CombMultiArgs ma{};
    ma.nsum = (int)n;
    ma.out_stride = c->words(lmin) * (size_t)B;
    for (size_t u = 0; u < terms.size(); ++u) {
        const ckks_ct *Ti = pb.T[terms[u]].get();
        if (Ti->B != B) return false;
        const double sc = (c->ladder[lmin - 1] * (double)c->q[lmin]) / Ti->scale;
        if (u > 0 && !scales_match(scale, Ti->scale * sc)) fail(CKKS_E_SCALE, "scale mismatch");
        ma.c.x[u] = Ti->buf.p;
        ma.c.member_stride[u] = (size_t)2 * (Ti->level + 1) * N;
        ma.c.poly_stride[u] = (size_t)(Ti->level + 1) * N;
        for (size_t t = 0; t < n; ++t) {
            const double kd = std::rint(cfs[t][terms[u]] * sc);
            if (!(std::fabs(kd) < 4.0e18)) fail(CKKS_E_RANGE, "constant out of range");
            ma.k[t][u] = (int64_t)kd;
        }
    }
    ma.c.nterm = (int)terms.size();
    // one launch: the first term of the first sum opens it; every further term adds one read
    // (the terms are read once for all sums) and every further sum one write
    for (size_t t = 0; t < n; ++t)
        for (size_t u = 0; u < terms.size(); ++u) trace_op(c, t == 0 && u == 0 ? "lincomb" : "lincomb_term", lmin, B);
    Ct acc = ct_new(c, lmin, scale, (int)n * B);
    gpu::lincomb_multi(c->T, acc->buf.p, ma, lmin + 1, B, map_q(0, lmin + 1), c->stream);
    std::shared_ptr<ckks_ct> rs(op_rescale(c, acc.get()).release());
    for (size_t t = 0; t < n; ++t) {
        Ct v = ct_view(c, rs, (int)t * B, B, rs->scale);
        out[t] = op_add_const(c, v.get(), cfs[t][0]);
    }
    return true;
}

// Several trees of the same height k at once (the quotient and remainder
// parts of one split are evaluated side by side): every tree's result is the
// recursive split p = q T_M + r of the coefficients, computed op for op as
// one tree alone would, with the products q T_M of all trees at one height
// sharing launch sequences.  D[t] is tree t's level budget below T_1 (D >= k):
// a tree ends in a baby-step sum when k <= b and its degree is at most
// 2^(D-1) (each T_i it combines then sits at most D-1 levels down and the
// sum takes one more); otherwise it is split by T_(2^(k-1)), the quotient
// with budget D-1, the remainder with D.  Only the leading quotient chain of
// a polynomial has D = k, so it alone is split below the baby-step height,
// and degree d takes bit_length(d) levels (the depth the paper states).
std::vector<Ct> cheb_trees(ckks_ctx *c, PowerBasis &pb, const std::vector<std::vector<double>> &cfs,
                           const std::vector<int> &D, int k, int b) {
    const size_t n = cfs.size();
    std::vector<Ct> out(n);
    std::vector<size_t> leaf, rest;
    for (size_t t = 0; t < n; ++t) {
        const int deg = (int)cfs[t].size() - 1;
        if (k <= b && deg <= (1 << (D[t] - 1))) leaf.push_back(t);
        else rest.push_back(t);
    }
    if (!leaf.empty()) {
        std::vector<std::vector<double>> lc;
        for (size_t t : leaf) lc.push_back(cfs[t]);
        std::vector<Ct> lo(lc.size());
        if (!baby_sums_together(c, pb, lc, lo))
            for (size_t u = 0; u < lc.size(); ++u) lo[u] = baby_sum(c, pb, lc[u]);
        for (size_t u = 0; u < leaf.size(); ++u) out[leaf[u]] = std::move(lo[u]);
    }
    if (rest.empty()) return out;
    const int M = 1 << (k - 1);
    std::vector<std::vector<double>> sub;
    std::vector<int> subD;
    std::vector<int> qi(n, -1), ri(n, -1);
    for (size_t t : rest) {
        const std::vector<double> &cf = cfs[t];
        const int deg = (int)cf.size() - 1;
        if (deg < M) {   // no split at this height
            ri[t] = (int)sub.size();
            sub.push_back(cf);
            subD.push_back(D[t]);
            continue;
        }
        const int dq = deg - M;
        std::vector<double> qc(dq + 1), rc(cf.begin(), cf.begin() + M);
        qc[0] = cf[M];
        for (int j = 1; j <= dq; ++j) qc[j] = 2.0 * cf[M + j];
        for (int j = 1; j <= dq; ++j) rc[M - j] = cf[M - j] - cf[M + j];
        qi[t] = (int)sub.size();
        sub.push_back(std::move(qc));
        subD.push_back(D[t] - 1);
        ri[t] = (int)sub.size();
        sub.push_back(std::move(rc));
        subD.push_back(D[t]);
    }
    std::vector<Ct> S = cheb_trees(c, pb, sub, subD, k - 1, b);
    std::vector<std::pair<const ckks_ct *, const ckks_ct *>> pairs;
    for (size_t t : rest)
        if (qi[t] >= 0) pairs.emplace_back(S[qi[t]].get(), pb.get(M));
    std::vector<Ct> P = mult_aligned_many(c, pairs);
    size_t j = 0;
    for (size_t t : rest) {
        if (qi[t] < 0) {
            out[t] = std::move(S[ri[t]]);
            continue;
        }
        out[t] = addsub_aligned(c, P[j].get(), S[ri[t]].get(), false);
        ++j;
    }
    return out;
}
Ct cheb_tree(ckks_ctx *c, PowerBasis &pb, const std::vector<double> &cf, int k, int b) {
    std::vector<Ct> r = cheb_trees(c, pb, {cf}, {k}, k, b);
    return std::move(r[0]);
}

int bit_length(int d) {
    int m = 0;
    while (d >> m) ++m;
    return m;
}

Ct op_cheb(ckks_ctx *c, const ckks_ct *x, const std::vector<double> &cf, double a, double b) {
    const int d = (int)cf.size() - 1;
    if (d < 1) fail(CKKS_E_PARAM, "degree must be >= 1");
    Ct t;
    if (a == -1.0 && b == 1.0) {
        t = ct_borrow(x, x->scale);   // x outlives the evaluation
    } else {
        if (x->level < 1) fail(CKKS_E_LEVEL, "no level for the affine map");
        double al = 2.0 / (b - a);
        double be = -(a + b) / (b - a);
        Ct m = op_mul_const_down(c, x, al);
        t = op_add_const(c, m.get(), be);
    }
    const int m = bit_length(d), bb = (m + 1) / 2;
    PowerBasis pb{c, {}};
    pb.T.resize((1 << m) + 1);
    pb.T[1] = std::move(t);
    std::vector<int> want;
    for (int i = 2; i < (1 << bb) && i <= d; ++i) want.push_back(i);
    for (int k = bb; k < m; ++k) want.push_back(1 << k);
    pb.ensure(want);
    return cheb_tree(c, pb, cf, m, bb);
}

// One Newton step y' = c15 y - (x/2 * y) * y^2 at c = min(l_x, l_y) (c15 =
// 1.5: the step of §2.2; the last step of a pre-normalised chain passes
// 1.5 / sqrt(B) with x/2 declared as x sqrt(B) / (2B)).  With raw_x the x
// operand is only limb-dropped (it keeps its own, larger scale); c15 y is
// encoded to land exactly on the scale of the product term.
Ct op_newton(ckks_ctx *c, const ckks_ct *y, const ckks_ct *half_x, bool raw_x, double c15 = 1.5) {
    const int lc = std::min(y->level, half_x->level);
    if (lc < 2) fail(CKKS_E_LEVEL, "Newton step needs 2 levels");
    Ct xa = raw_x ? op_drop(c, half_x, lc) : op_level_to(c, half_x, lc);
    Ct ya = op_level_to(c, y, lc);
    // tmp_beta = ct_x * y and y^2, both from y at the step's level: one wave
    std::vector<Ct> uv = mult_aligned_many(c, {{xa.get(), ya.get()}, {ya.get(), ya.get()}});
    xa.reset();
    ya.reset();
    Ct u = std::move(uv[0]), v = std::move(uv[1]);
    Ct w = mult_rs(c, u.get(), v.get());            // tmp_beta * y^2
    u.reset();
    v.reset();
    double sc = (w->scale * (double)c->q[lc - 1]) / y->scale;
    Ct tm = op_lincomb(c, {y}, {c15}, {sc}, lc - 1);   // tmp_alpha = 1.5 y (limbs to lc-1) on scale(w)
    Ct ta = op_rescale(c, tm.get());
    return op_addsub(c, ta.get(), w.get(), true);
}

// ---------------------------------------------------------------------------
// Bootstrapping (ModRaise, CoeffToSlot, EvalMod, SlotToCoeff)
// ---------------------------------------------------------------------------
// levels op_cheb consumes for degree d on [-1, 1] (another interval adds the
// affine map's level): the bit length of d
int cheb_depth(int d) { return bit_length(d); }

void upload_signed_ntt(ckks_ctx *c, u64 *dst, const int64_t *src_host, int nlimb, const LimbMap &m);

// NTT of X^k (0 <= k < 2N) over q_0..q_L, cached
const u64 *mono_table(ckks_ctx *c, int k) {
    auto it = c->mono.find(k);
    if (it != c->mono.end()) return it->second.p;
    const int nq = c->L + 1;
    std::vector<int64_t> coef(c->N, 0);
    coef[k % c->N] = k < c->N ? 1 : -1;   // X^N = -1
    Buf t(c->pool.get(), (size_t)nq * c->N);
    upload_signed_ntt(c, t.p, coef.data(), nq, map_q(0, nq));
    const u64 *p = t.p;
    c->mono.emplace(k, std::move(t));
    return p;
}

Ct op_mul_monomial(ckks_ctx *c, const ckks_ct *a, int k) {
    k %= 2 * c->N;
    if (k < 0) k += 2 * c->N;
    const u64 *tab = mono_table(c, k);
    trace_op(c, "mul_scalar", a->level, a->B);
    Ct r = ct_new(c, a->level, a->scale, a->B);
    gpu::MacArgs ma{};
    ma.nterm = 1;
    ma.pt[0] = tab;
    ma.x[0] = a->buf.p;
    gpu::pt_mac(c->T, r->buf.p, ma, a->level + 1, 2 * a->B, map_q(0, a->level + 1), c->stream);
    return r;
}

// residues mod q_0 lifted to the centred range, reduced mod q_0..q_L
Ct op_mod_raise(ckks_ctx *c, const ckks_ct *a) {
    if (!c->bts) fail(CKKS_E_NOKEY, "bootstrapping not set up");
    const int L = c->L, B = a->B, np2 = 2 * B;
    const size_t N = c->N;
    trace_op(c, "mod_raise", L, B);
    Ct r = ct_new(c, L, 2.0 * (double)c->q[0] * c->bts->K, B);
    Buf t(c->pool.get(), (size_t)np2 * N);
    ntt_oop_p(c, t.p, a->buf.p, (size_t)(a->level + 1) * N, 1, np2, map_q(0, 1), true);
    if (c->logN == 16) {
        gpu::NttLift lf{t.p, N, 0};   // the lift fused into the transform's first pass
        ProfScope ps(c, "ntt", 16.0 * (double)(L + 1) * np2 * N);
        gpu::ntt16_fwd_fused(c->T, r->buf.p, &lf, nullptr, L + 1, np2, map_q(0, L + 1), c->stream);
        return r;
    }
    gpu::rescale_lift(c->T, r->buf.p, t.p, 0, L + 1, np2, N, c->stream);
    ntt_p(c, r->buf.p, L + 1, np2, map_q(0, L + 1), false);
    return r;
}

// sum_i rot_{g i s}( sum_b P_{i,b} * rot_{b s}(x) ), then one rescale
Ct op_lt(ckks_ctx *c, const ckks_ct *x, const LtStage &st) {
    if (x->level != st.level) fail(CKKS_E_LEVEL, "slot transform at the wrong level");
    const int n = c->N / 2, nq = x->level + 1, B = x->B;
    // baby steps: every used b, rotated by b * stride, from one hoisted ModUp
    std::vector<int> bs;
    for (int b : st.baby)
        if (b != 0 && std::find(bs.begin(), bs.end(), b) == bs.end()) bs.push_back(b);
    std::sort(bs.begin(), bs.end());
    std::vector<int> ks;
    for (int b : bs) ks.push_back(b * st.stride);
    std::vector<Ct> rot = op_rotate_hoisted(c, x, ks);
    std::map<int, Ct> R;
    for (size_t t = 0; t < bs.size(); ++t) R[bs[t]] = std::move(rot[t]);
    // inner sums of every giant step into one buffer [giant][B][2][nq][N]:
    // the rotated giants first (their ModUp is one batch), giant 0 last
    std::vector<int> gis;
    for (int gi : st.giant)
        if (std::find(gis.begin(), gis.end(), gi) == gis.end()) gis.push_back(gi);
    std::stable_partition(gis.begin(), gis.end(), [](int gi) { return gi != 0; });
    const size_t N = c->N, member = (size_t)2 * nq * N, gstride = member * B;
    Buf inner(c->pool.get(), gstride * gis.size());
    if (bs.size() + 1 <= (size_t)gpu::kMaxBaby && gis.size() <= (size_t)gpu::kMaxGiant) {
        // every inner sum in one pass over the babies
        gpu::GiantArgs ga{};
        ga.nb = (int)bs.size() + 1;
        ga.ng = (int)gis.size();
        ga.x[0] = x->buf.p;
        for (size_t t = 0; t < bs.size(); ++t) ga.x[t + 1] = R[bs[t]]->buf.p;
        for (size_t k = 0; k < gis.size(); ++k) {
            for (size_t t = 0; t < st.giant.size(); ++t) {
                if (st.giant[t] != gis[k]) continue;
                const int b = st.baby[t];
                const int bi = b == 0 ? 0 : 1 + (int)(std::find(bs.begin(), bs.end(), b) - bs.begin());
                if (ga.pt[k][bi]) fail(CKKS_E_PARAM, "repeated diagonal in a slot transform");
                ga.pt[k][bi] = st.pt[t].p;
            }
            trace_op(c, "mul_plain", x->level, B);
        }
        gpu::pt_mac_giants(c->T, inner.p, gstride, ga, nq, B, map_q(0, nq), c->stream);
    } else for (size_t k = 0; k < gis.size(); ++k) {
        gpu::MacArgs ma{};
        for (size_t t = 0; t < st.giant.size(); ++t) {
            if (st.giant[t] != gis[k]) continue;
            if (ma.nterm >= gpu::kMaxMac) fail(CKKS_E_PARAM, "too many baby steps");
            const int b = st.baby[t];
            ma.pt[ma.nterm] = st.pt[t].p;
            ma.x[ma.nterm] = b == 0 ? x->buf.p : R[b]->buf.p;
            ++ma.nterm;
        }
        trace_op(c, "mul_plain", x->level, B);
        gpu::pt_mac(c->T, inner.p + k * gstride, ma, nq, 2 * B, map_q(0, nq), c->stream);
    }
    const size_t nrot = gis.size() - (gis.back() == 0 ? 1 : 0);
    if (nrot > 0) {
        std::vector<RotJob> jobs;
        for (size_t k = 0; k < nrot; ++k) {
            const long long steps = ((long long)st.g * gis[k] * st.stride) % n;
            const int g = galois_rot(c, (int)steps);
            auto it = c->rot.find(g);
            if (it == c->rot.end()) fail(CKKS_E_NOKEY, "missing Galois key");
            trace_op(c, "rotate", x->level, B);
            jobs.push_back(RotJob{&it->second, perm_for(c, g), (int)(k * B), nullptr, inner.p + k * gstride});
        }
        ModUp mu;
        {
            ProfScope ps(c, "keyswitch", 8.0 * (double)N * nrot * B * nq);
            modup(c, x->level, inner.p + (size_t)nq * N, member, (int)(nrot * B), mu);
        }
        // the rotated giants' inner products summed over Q_l and P (A), their
        // rotated c0 and giant 0's inner sum over Q_l (E); then one ModDown by
        // P q_l of A + P E: the rotations' ModDowns, their sum and the
        // rescale in one
        const int l = x->level, K = c->K, ne = nq + K;
        const int beta = (nq + c->alpha - 1) / c->alpha;
        ProfScope ps(c, "keyswitch", 8.0 * (double)N * ((double)nrot * 2.0 * beta * ne + 2.0 * B * l));
        Pool *Pl = c->pool.get();
        Buf A(Pl, (size_t)B * 2 * ne * N), E(Pl, (size_t)B * 2 * nq * N);
        const u64 *g0 = gis.size() > nrot ? inner.p + nrot * gstride : nullptr;
        // the summing inner product adds njob * ndig products of words below
        // the primes in 128 bits before one reduction: at most
        // c->sum_terms terms per launch (their sum stays below 2^127)
        if (mu.ia.ndig > c->sum_terms) fail(CKKS_E_PARAM, "too many digits for a summed inner product");
        const size_t per = (size_t)std::max(1, std::min(gpu::kMaxJobs, c->sum_terms / mu.ia.ndig));
        for (size_t j0 = 0; j0 < jobs.size(); j0 += per) {
            const int nj = (int)std::min<size_t>(per, jobs.size() - j0);
            gpu::KsJobs kj{};
            gpu::FinishJobs fj{};
            kj.njob = nj;
            kj.B = B;
            for (int t = 0; t < nj; ++t) {
                const RotJob &jb = jobs[j0 + t];
                kj.ct0[t] = jb.ct0;
                kj.key[t] = jb.key->k.p;
                kj.perm[t] = jb.perm;
                fj.add[t] = jb.add;
                fj.perm[t] = jb.perm;
            }
            gpu::key_inner_jobs_sum(c->T, A.p, mu.ia, kj, j0 > 0, c->stream);
            gpu::rot_c0_sum(c->T, fj, E.p, g0, j0 > 0, nq, nj, B, map_q(0, nq), c->stream);
        }
        trace_op(c, "rescale", l, B);
        Ct r = ct_new(c, l - 1, (x->scale * st.sd) / (double)c->q[l], B);
        moddown_rescale(c, l, A.p, E.p, 2 * B, r->buf.p);
        return r;
    }
    // giant 0 alone: its inner sum, rescaled
    Ct acc = ct_new(c, x->level, x->scale * st.sd, B);
    hipchk(hipMemcpyAsync(acc->buf.p, inner.p, gstride * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
    return op_rescale(c, acc.get());
}

Ct op_coeff_to_slot(ckks_ctx *c, const ckks_ct *a) {
    if (!c->bts) fail(CKKS_E_NOKEY, "bootstrapping not set up");
    if (a->level != c->L) fail(CKKS_E_LEVEL, "CoeffToSlot expects a ModRaised ciphertext");
    Ct x = op_lt(c, a, c->bts->cts[0]);
    x = op_lt(c, x.get(), c->bts->cts[1]);
    return op_lt(c, x.get(), c->bts->cts[2]);
}
Ct op_slot_to_coeff(ckks_ctx *c, const ckks_ct *a) {
    if (!c->bts) fail(CKKS_E_NOKEY, "bootstrapping not set up");
    if (a->level != c->shape.l_after + 3) fail(CKKS_E_LEVEL, "SlotToCoeff expects the EvalMod output level");
    Ct x = op_lt(c, a, c->bts->stc[0]);
    x = op_lt(c, x.get(), c->bts->stc[1]);
    return op_lt(c, x.get(), c->bts->stc[2]);
}
Ct op_eval_mod(ckks_ctx *c, const ckks_ct *u) {
    if (!c->bts) fail(CKKS_E_NOKEY, "bootstrapping not set up");
    Ct y = op_cheb(c, u, c->bts->cf, -1.0, 1.0);
    for (int k = 0; k < c->bts->r; ++k) {
        Ct sq = mult_rs(c, y.get(), y.get());
        y = op_mul_int_add_const(c, sq.get(), 2, -1.0);   // cos 2t = 2 cos^2 t - 1
    }
    return y;
}

// two ciphertext objects of equal level, scale and B as one batch of 2B
Ct concat2(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b) {
    const size_t w = c->words(a->level) * a->B;
    Ct r = ct_new(c, a->level, a->scale, 2 * a->B);
    hipchk(hipMemcpyAsync(r->buf.p, a->buf.p, w * 8, hipMemcpyDeviceToDevice, c->stream), "concat");
    hipchk(hipMemcpyAsync(r->buf.p + w, b->buf.p, w * 8, hipMemcpyDeviceToDevice, c->stream), "concat");
    return r;
}
Ct half_of(ckks_ctx *c, const ckks_ct *ab, int which) {
    const int B = ab->B / 2;
    const size_t w = c->words(ab->level) * B;
    Ct r = ct_new(c, ab->level, ab->scale, B);
    hipchk(hipMemcpyAsync(r->buf.p, ab->buf.p + (size_t)which * w, w * 8, hipMemcpyDeviceToDevice, c->stream),
           "split");
    return r;
}

Ct op_bootstrap(ckks_ctx *c, const ckks_ct *a, int64_t bound) {
    if (!c->bts) fail(CKKS_E_NOKEY, "bootstrapping not set up");
    if (bound < 1) fail(CKKS_E_PARAM, "message bound must be >= 1");
    const int N = c->N;
    const double s0 = std::ldexp((double)c->q[0], -5);
    const double Fd = std::rint(s0 / (a->scale * (double)bound));
    if (!(Fd >= 1.0 && Fd < 1099511627776.0)) fail(CKKS_E_RANGE, "input scale out of range for bootstrapping");
    trace_op(c, "bootstrap", a->level, a->B);
    struct Mute {
        ckks_ctx *c;
        explicit Mute(ckks_ctx *c_) : c(c_) { ++c->trace_mute; }
        ~Mute() { --c->trace_mute; }
    } mute(c);
    Ct a0 = op_drop(c, a, 0);
    Ct aF = op_mul_int(c, a0.get(), (int64_t)Fd, a0->scale);
    a0.reset();
    Ct raised = op_mod_raise(c, aF.get());
    aF.reset();
    Ct y = op_coeff_to_slot(c, raised.get());
    raised.reset();
    Ct yc = op_automorphism(c, y.get(), 2 * N - 1);
    Ct sum = op_addsub(c, y.get(), yc.get(), false);
    Ct dif = op_addsub(c, y.get(), yc.get(), true);
    y.reset();
    yc.reset();
    Ct im = op_mul_monomial(c, dif.get(), 3 * N / 2);
    dif.reset();
    Ct both = concat2(c, sum.get(), im.get());
    sum.reset();
    im.reset();
    Ct e = op_eval_mod(c, both.get());
    both.reset();
    std::shared_ptr<ckks_ct> es(e.release());   // the real and imaginary halves as views
    Ct er = ct_view(c, es, 0, es->B / 2, es->scale), ei = ct_view(c, es, es->B / 2, es->B / 2, es->scale);
    es.reset();
    Ct eii = op_mul_monomial(c, ei.get(), N / 2);
    ei.reset();
    Ct w = op_addsub(c, er.get(), eii.get(), false);
    er.reset();
    eii.reset();
    Ct z = op_slot_to_coeff(c, w.get());
    return op_mul_int(c, z.get(), bound, z->scale * (((a->scale * Fd) * (double)bound) / s0));
}

void bts_setup(ckks_ctx *c, double K, int r, int deg) {
    const hm::ChainShape &sh = c->shape;
    if (sh.n_evm <= 0) fail(CKKS_E_PARAM, "chain has no bootstrapping levels");
    if (sh.n_stc != 3 || sh.n_cts != 3 || deg < 2 || r < 0 || !(K > 1) || sh.n_evm != cheb_depth(deg) + r)
        fail(CKKS_E_PARAM, "bootstrapping configuration does not match the chain");
    std::unique_ptr<BtsPlan> b(new BtsPlan);
    b->K = K;
    b->r = r;
    b->deg = deg;
    b->cf.resize(deg + 1);
    hm::cheb_cosmod(deg, K, std::ldexp(1.0, r), b->cf.data());
    const int logn = c->logN - 1, L = c->L, A = sh.l_after;
    const double s0 = std::ldexp((double)c->q[0], -5);
    int sizes[3], top = logn;
    for (int i = 0; i < 3; ++i) sizes[i] = logn / 3 + (i < logn % 3 ? 1 : 0);
    // Nominal scale chains.  CoeffToSlot: from the ModRaise scale 2 q_0 K to
    // S_{L-3}; SlotToCoeff: from S_{A+3} (the EvalMod output) to S_A.  With
    // f = cbrt(end / start) the targets are start f, start f f, end; stage t
    // at level lv uses s_d = (target q_lv) / s and leaves s <- (s s_d) / q_lv.
    double sd[2][3];
    for (int pass = 0; pass < 2; ++pass) {
        int lv = pass == 0 ? L : A + 3;
        double s = pass == 0 ? 2.0 * (double)c->q[0] * K : c->ladder[A + 3];
        const double end = pass == 0 ? c->ladder[L - 3] : c->ladder[A];
        const double f = std::cbrt(end / s);
        double tg[3];
        tg[0] = s * f;
        tg[1] = tg[0] * f;
        tg[2] = end;
        for (int t = 0; t < 3; ++t, --lv) {
            sd[pass][t] = (tg[t] * (double)c->q[lv]) / s;
            s = (s * sd[pass][t]) / (double)c->q[lv];
        }
    }
    auto build = [&](LtStage &st, const std::vector<int> &ks, bool inverse, bool carry_const, int level,
                     double scale) {
        hm::LtGroupPlan gp;
        if (!hm::lt_group(c->logN, ks.data(), (int)ks.size(), inverse, c->q[0], carry_const ? s0 : 0.0, scale, gp))
            fail(CKKS_E_RANGE, "diagonal plaintext out of range");
        st.level = level;
        st.stride = gp.stride;
        st.g = gp.g;
        st.sd = scale;
        const int nq = level + 1;
        for (auto &t : gp.terms) {
            st.giant.push_back(t.giant);
            st.baby.push_back(t.baby);
            Buf pt(c->pool.get(), (size_t)nq * c->N);
            upload_signed_ntt(c, pt.p, t.coef.data(), nq, map_q(0, nq));
            st.pt.push_back(std::move(pt));
        }
    };
    for (int i = 0; i < 3; ++i) {
        std::vector<int> ks, kr;
        for (int t = 0; t < sizes[i]; ++t) ks.push_back(top - t);
        for (int t = 0; t < sizes[i]; ++t) kr.push_back(top - sizes[i] + 1 + t);
        build(b->cts[i], ks, true, false, L - i, sd[0][i]);
        build(b->stc[2 - i], kr, false, i == 2, A + 3 - (2 - i), sd[1][2 - i]);
        top -= sizes[i];
    }
    c->bts = std::move(b);
}

std::vector<int> bts_rotations(const ckks_ctx *c) {
    if (!c->bts) fail(CKKS_E_NOKEY, "bootstrapping not set up");
    const int n = c->N / 2;
    std::vector<char> seen(n, 0);
    const LtStage *all[6] = {&c->bts->cts[0], &c->bts->cts[1], &c->bts->cts[2],
                             &c->bts->stc[0], &c->bts->stc[1], &c->bts->stc[2]};
    for (const LtStage *st : all)
        for (size_t t = 0; t < st->giant.size(); ++t) {
            const long long kb = ((long long)st->baby[t] * st->stride) % n;
            const long long kg = (((long long)st->g * st->giant[t] * st->stride) % n + n) % n;
            if (kb) seen[kb] = 1;
            if (kg) seen[kg] = 1;
        }
    std::vector<int> out;
    for (int k = 1; k < n; ++k)
        if (seen[k]) out.push_back(k);
    return out;
}

// The context's Chebyshev coefficients of 1/sqrt on [a, b] at degree d (the
// interpolation of the host's own quad-precision routine, computed on the
// first request and kept; at most 64 intervals are kept, then the cache starts
// over).
static std::vector<double> cheb_coeffs_invsqrt(ckks_ctx *c, int d, double a, double b) {
    const auto key = std::make_tuple(d, a, b);
    auto it = c->cheb_cf.find(key);
    if (it != c->cheb_cf.end()) return it->second;
    std::vector<double> cf(d + 1);
    hm::cheb_invsqrt(d, a, b, cf.data());
    if (c->cheb_cf.size() >= 64) c->cheb_cf.clear();
    c->cheb_cf.emplace(key, cf);
    return cf;
}

// CryptoInvSqrt with the bootstrapping policy: Pre-BTS of x (paper's c = 1)
// when asked for (opts.pre_bts) or when x cannot carry the Chebyshev step or
// ct_x; otherwise x is never bootstrapped.  Lazy bootstrapping of y before a Newton step that lacks 2
// levels (or right after the Chebyshev step with `literal`).
Ct op_invsqrt(ckks_ctx *c, const ckks_ct *x0, int degree, int iters, const ckks_invsqrt_opts &o) {
    if (degree < 1 || iters < 0) fail(CKKS_E_PARAM, "bad degree / iterations");
    if (!(o.a > 0) || !(o.b > o.a)) fail(CKKS_E_PARAM, "bad interval");
    if (!(o.B >= 0) || !std::isfinite(o.B)) fail(CKKS_E_PARAM, "bad pre-normalisation constant");
    // pre-normalisation: u = x / Bn on [an, bn]; output scaled by kappa
    const double Bn = o.B > 0 ? o.B : 1.0, an = o.a / Bn, bn = o.b / Bn, kappa = 1.0 / std::sqrt(Bn);
    const int64_t My = o.bts_bound > 0 ? o.bts_bound : 16 * (int64_t)std::ceil(1.0 / std::sqrt(an));
    const ckks_ct *x = x0;
    Ct xb;
    // x holds (input) / sx: sx = B once the input has been divided by B ahead
    // of a Pre-BTS (the bootstrap then sees a message bounded by b/B, which the
    // input scale leaves room for where b itself would not), else 1
    double sx = 1.0;
    if (o.pre_bts || x->level < cheb_depth(degree) + 1 || x->level < 3) {
        if (!c->bts) {
            if (o.pre_bts) fail(CKKS_E_NOKEY, "Pre-BTS needs bootstrapping");
            if (x->level < 2) fail(CKKS_E_LEVEL, "input needs at least 2 levels");
        } else {
            Ct xn;
            if (Bn > 1.0) {
                xn = op_mul_const_down(c, x, 1.0 / Bn);
                x = xn.get();
                sx = Bn;
            }
            xb = op_bootstrap(c, x, 16 * (int64_t)std::ceil(o.b / sx));
            x = xb.get();
        }
    }
    std::vector<double> cf = cheb_coeffs_invsqrt(c, degree, an, bn);
    if (iters == 0)
        for (double &v : cf) v *= kappa;   // no Newton step to carry the scale-back
    Ct cx = op_mul_const_down(c, x, 0.5 * sx / Bn);
    // affine map from [a/sx, b/sx] (the interval of what x holds): t(x) = t(u) on [an, bn]
    Ct y = op_cheb(c, x, cf, o.a / sx, o.b / sx);
    if (o.literal) y = op_bootstrap(c, y.get(), My);
    for (int i = 0; i < iters; ++i) {
        if (y->level < 2) {
            if (cx->level < 2) fail(CKKS_E_LEVEL, "x has too few levels for Newton");
            y = op_bootstrap(c, y.get(), My);
        }
        if (i == iters - 1) {
            // last step: u/2 = x/(2B) straight from the input as an exact
            // change of scale, with the scale-back kappa = 1/sqrt(B) folded
            // in: the x operand declared as kappa x / (2B), the constant
            // 1.5 kappa
            Ct xr = ct_borrow(x, x->scale * (2.0 * (Bn / sx) * std::sqrt(Bn)));
            y = op_newton(c, y.get(), xr.get(), true, 1.5 * kappa);
        } else {
            y = op_newton(c, y.get(), cx.get(), false);
        }
    }
    return y;
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
void upload_signed_ntt(ckks_ctx *c, u64 *dst, const int64_t *src_host, int nlimb, const LimbMap &m) {
    Buf tmp(c->pool.get(), c->N);
    hipchk(hipMemcpyAsync(tmp.p, src_host, c->N * 8, hipMemcpyHostToDevice, c->stream), "upload");
    gpu::signed_to_residues(c->T, dst, (const int64_t *)tmp.p, nlimb, m, c->stream);
    gpu::ntt(c->T, dst, nlimb, 1, m, false, c->stream);
    hipchk(hipStreamSynchronize(c->stream), "sync");   // host buffer reuse
}

void make_switch_key(ckks_ctx *c, uint64_t seed, int galois, const u64 *sprime, SwitchKey &out) {
    const size_t N = c->N;
    const int np = c->np;
    out.k = Buf(c->pool.get(), (size_t)c->dnum * 2 * np * N);
    std::vector<u64> a((size_t)np * N);
    std::vector<int64_t> e(N);
    LimbMap all = map_q(0, np);
    Buf eN(c->pool.get(), (size_t)np * N);
    LimbConsts pm{};
    std::vector<int> pidx;
    for (int k = 0; k < c->K; ++k) pidx.push_back(c->L + 1 + k);
    for (int i = 0; i <= c->L; ++i) {
        pm.v[i] = prod_mod(c, pidx, -1, c->q[i]);
        pm.sh[i] = shoup(pm.v[i], c->q[i]);
    }
    for (int j = 0; j < c->dnum; ++j) {
        u64 *b = out.k.p + ((size_t)j * 2 + 0) * np * N;
        u64 *ak = out.k.p + ((size_t)j * 2 + 1) * np * N;
        hm::Shake256 xa(seed, hm::stream_tag(hm::kKeyA, galois, j));
        for (int i = 0; i < np; ++i) hm::uniform_residues(xa, c->q[i], c->N, a.data() + (size_t)i * N);
        hipchk(hipMemcpyAsync(ak, a.data(), a.size() * 8, hipMemcpyHostToDevice, c->stream), "key upload");
        hm::Shake256 xe(seed, hm::stream_tag(hm::kKeyE, galois, j));
        hm::gaussian(xe, c->cdt, c->N, e.data());
        upload_signed_ntt(c, eN.p, e.data(), np, all);
        std::vector<uint8_t> flag(np, 0);
        for (int i = j * c->alpha; i < std::min((j + 1) * c->alpha, c->L + 1); ++i) flag[i] = 1;
        gpu::key_combine(c->T, b, ak, c->sk.p, eN.p, sprime, pm, flag.data(), np, all, c->stream);
    }
    hipchk(hipStreamSynchronize(c->stream), "key sync");
}

// every level's key-switching conversion tables (ModUp per digit, ModDown),
// so that key switches issued later allocate no tables
void build_ks_tables(ckks_ctx *c) {
    for (int l = 0; l <= c->L; ++l) {
        const int beta = (l + 1 + c->alpha - 1) / c->alpha;
        for (int j = 0; j < beta; ++j) modup_table(c, l, j);
        moddown_table(c, l);
    }
}

void keygen(ckks_ctx *c, uint64_t seed, const int32_t *gal, uint32_t ng) {
    const size_t N = c->N;
    const int np = c->np;
    Pool *P = c->pool.get();
    std::vector<int8_t> s(N);
    hm::Shake256 xs(seed, hm::stream_tag(hm::kSecret, 0, 0));
    if (c->prm.hamming_weight > 0) hm::hamming_ternary(xs, c->N, (int)c->prm.hamming_weight, s.data());
    else hm::ternary(xs, c->N, s.data());
    std::vector<int64_t> s64(s.begin(), s.end());
    c->sk = Buf(P, (size_t)np * N);
    upload_signed_ntt(c, c->sk.p, s64.data(), np, map_q(0, np));
    // public key over q_0..q_L
    const int nq = c->L + 1;
    c->pk = Buf(P, 2 * (size_t)nq * N);
    std::vector<u64> a((size_t)nq * N);
    hm::Shake256 xa(seed, hm::stream_tag(hm::kPkA, 0, 0));
    for (int i = 0; i < nq; ++i) hm::uniform_residues(xa, c->q[i], c->N, a.data() + (size_t)i * N);
    u64 *pk1 = c->pk.p + (size_t)nq * N;
    hipchk(hipMemcpyAsync(pk1, a.data(), a.size() * 8, hipMemcpyHostToDevice, c->stream), "pk upload");
    std::vector<int64_t> e(N);
    hm::Shake256 xe(seed, hm::stream_tag(hm::kPkE, 0, 0));
    hm::gaussian(xe, c->cdt, c->N, e.data());
    Buf eN(P, (size_t)nq * N);
    upload_signed_ntt(c, eN.p, e.data(), nq, map_q(0, nq));
    LimbConsts none{};
    gpu::key_combine(c->T, c->pk.p, pk1, c->sk.p, eN.p, nullptr, none, nullptr, nq, map_q(0, nq), c->stream);
    // relinearisation key: s' = s^2
    Buf s2(P, (size_t)np * N);
    gpu::mul_pointwise(c->T, s2.p, c->sk.p, c->sk.p, np, 1, map_q(0, np), c->stream);
    make_switch_key(c, seed, 0, s2.p, c->relin);
    c->rot.clear();
    for (uint32_t r = 0; r < ng; ++r) {
        int g = gal[r];
        if (g <= 0 || g >= 2 * c->N || (g & 1) == 0) fail(CKKS_E_PARAM, "bad Galois element");
        if (c->rot.count(g)) continue;
        const int32_t *perm = perm_for(c, g);
        gpu::permute(c->T, s2.p, c->sk.p, perm, np, 1, c->stream);
        make_switch_key(c, seed, g, s2.p, c->rot[g]);
    }
    build_ks_tables(c);
    c->have_keys = true;
}

// host stage of encryption: encoded message + sampled randomness
struct EncHost {
    std::vector<int64_t> v, e0m, e1;
    bool ok = true;
};
void enc_host(const ckks_ctx *c, const double *x, uint32_t n, double scale, uint64_t seed, EncHost &h) {
    const size_t N = c->N;
    std::vector<int64_t> m(N);
    h.ok = hm::encode(c->logN, x, nullptr, n, scale, m.data());
    std::vector<int8_t> v(N);
    h.e0m.assign(N, 0);
    h.e1.assign(N, 0);
    hm::Shake256 xv(seed, hm::stream_tag(hm::kEncV, 0, 0));
    hm::ternary(xv, c->N, v.data());
    hm::Shake256 x0(seed, hm::stream_tag(hm::kEncE0, 0, 0));
    hm::gaussian(x0, c->cdt, c->N, h.e0m.data());
    hm::Shake256 x1(seed, hm::stream_tag(hm::kEncE1, 0, 0));
    hm::gaussian(x1, c->cdt, c->N, h.e1.data());
    for (size_t j = 0; j < N; ++j) h.e0m[j] += m[j];
    h.v.assign(v.begin(), v.end());
}
// device stage: ct0 = v pk0 + e0 + m, ct1 = v pk1 + e1 (NTT domain)
Ct enc_device(ckks_ctx *c, const EncHost &h, int level, double scale) {
    const size_t N = c->N;
    const int nq = level + 1;
    Pool *P = c->pool.get();
    Buf vN(P, (size_t)nq * N), a0(P, (size_t)nq * N), a1(P, (size_t)nq * N);
    LimbMap mq = map_q(0, nq);
    upload_signed_ntt(c, vN.p, h.v.data(), nq, mq);
    upload_signed_ntt(c, a0.p, h.e0m.data(), nq, mq);
    upload_signed_ntt(c, a1.p, h.e1.data(), nq, mq);
    Ct r = ct_new(c, level, scale);
    const u64 *pk0 = c->pk.p, *pk1 = c->pk.p + (size_t)(c->L + 1) * N;
    gpu::mul_add(c->T, poly(c, r.get(), 0), vN.p, pk0, a0.p, nq, mq, c->stream);
    gpu::mul_add(c->T, poly(c, r.get(), 1), vN.p, pk1, a1.p, nq, mq, c->stream);
    return r;
}

Ct op_encrypt(ckks_ctx *c, const double *x, uint32_t n, int level, double scale, uint64_t seed) {
    if (!c->have_keys) fail(CKKS_E_NOKEY, "no keys");
    if (level < 0 || level > c->L) fail(CKKS_E_LEVEL, "bad level");
    if (n > (uint32_t)c->N / 2) fail(CKKS_E_PARAM, "too many slots");
    EncHost h;
    enc_host(c, x, n, scale, seed, h);
    if (!h.ok) fail(CKKS_E_RANGE, "value out of range for encoding");
    return enc_device(c, h, level, scale);
}

void op_decrypt(ckks_ctx *c, const ckks_ct *ct, double *re, double *im) {
    if (!c->have_keys) fail(CKKS_E_NOKEY, "no keys");
    if (ct->B != 1) fail(CKKS_E_PARAM, "batched ciphertext object");
    const int nq = ct->level + 1;
    const size_t N = c->N;
    Buf m(c->pool.get(), (size_t)nq * N);
    gpu::decrypt_combine(c->T, m.p, poly(c, ct, 0), poly(c, ct, 1), c->sk.p, nq, map_q(0, nq), c->stream);
    gpu::ntt(c->T, m.p, nq, 1, map_q(0, nq), true, c->stream);
    std::vector<u64> host((size_t)nq * N);
    hipchk(hipMemcpyAsync(host.data(), m.p, host.size() * 8, hipMemcpyDeviceToHost, c->stream), "download");
    hipchk(hipStreamSynchronize(c->stream), "sync");
    hm::decode_residues(c->logN, host.data(), nq, c->q.data(), ct->scale, re, im);
}

}  // namespace

// A captured CryptoInvSqrt chain for inputs of one shape (level, scale, B).
struct ckks_graph {
    Ct in, out;
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    std::vector<void *> owned;
};

namespace {

void graph_free(ckks_ctx *c, ckks_graph *G) {
    if (G->ex) (void)hipGraphExecDestroy(G->ex);
    if (G->g) (void)hipGraphDestroy(G->g);
    G->out.reset();
    G->in.reset();
    c->pool->release_graph(G->owned);
    delete G;
}

// Capture: one eager run first (fills every first-use table and the pool's
// cache, so the captured run neither synchronises nor allocates device
// memory), then the same chain on a dedicated input under stream capture.
ckks_graph *graph_create(ckks_ctx *c, const ckks_ct *x, int degree, int iters, const ckks_invsqrt_opts &o) {
    {
        Ct warm = op_invsqrt(c, x, degree, iters, o);
    }
    hipchk(hipStreamSynchronize(c->stream), "sync");
    std::unique_ptr<ckks_graph> G(new ckks_graph);
    G->in = ct_copy(c, x);
    hipchk(hipStreamSynchronize(c->stream), "sync");
    // capture on a private stream (the context's stream may be the null
    // stream, which cannot be captured); replays go to the context's stream
    if (!c->cap_stream) hipchk(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
    hipStream_t user = c->stream;
    const bool prof = c->prof_on;
    c->prof_on = false;
    c->stream = c->cap_stream;
    c->pool->begin_capture();
    auto restore = [&] {
        c->stream = user;
        c->prof_on = prof;
    };
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        G->owned = c->pool->end_capture();
        restore();
        graph_free(c, G.release());
        fail(CKKS_E_DEVICE, "stream capture could not begin");
    }
    try {
        G->out = op_invsqrt(c, G->in.get(), degree, iters, o);
    } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(c->stream, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        G->owned = c->pool->end_capture();
        restore();
        graph_free(c, G.release());
        throw;
    }
    hipError_t e = hipStreamEndCapture(c->stream, &G->g);
    G->owned = c->pool->end_capture();
    restore();
    if (e != hipSuccess) {
        graph_free(c, G.release());
        fail(CKKS_E_DEVICE, "stream capture failed");
    }
    if (hipGraphInstantiate(&G->ex, G->g, nullptr, nullptr, 0) != hipSuccess) {
        graph_free(c, G.release());
        fail(CKKS_E_DEVICE, "graph instantiation failed");
    }
    return G.release();
}

Ct graph_run(ckks_ctx *c, ckks_graph *G, const ckks_ct *x) {
    if (x->level != G->in->level || x->scale != G->in->scale || x->B != G->in->B)
        fail(CKKS_E_PARAM, "input shape differs from the captured one");
    const size_t w = c->words(x->level) * x->B;
    hipchk(hipMemcpyAsync(G->in->buf.p, x->buf.p, w * 8, hipMemcpyDeviceToDevice, c->stream), "graph input");
    hipchk(hipGraphLaunch(G->ex, c->stream), "graph launch");
    Ct r = ct_new(c, G->out->level, G->out->scale, G->out->B);
    hipchk(hipMemcpyAsync(r->buf.p, G->out->buf.p, c->words(r->level) * r->B * 8, hipMemcpyDeviceToDevice, c->stream),
           "graph output");
    return r;
}

// C-ABI wrapper: run f, map exceptions to a status
template <class F>
ckks_status guard(ckks_ctx *c, F &&f) {
    try {
        f();
        return CKKS_OK;
    } catch (const Error &e) {
        if (c) c->err = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        return CKKS_E_OOM;
    } catch (const std::exception &e) {
        if (c) c->err = e.what();
        return CKKS_E_PARAM;
    }
}
template <class F>
ckks_status guard_out(ckks_ctx *c, ckks_ct **out, F &&f) {
    if (!out) {
        if (c) c->err = "null output pointer";
        return CKKS_E_PARAM;
    }
    *out = nullptr;
    return guard(c, [&] { *out = f().release(); });
}

}  // namespace

// ---------------------------------------------------------------------------
// The scratch array of the entry point that allocates nothing
// (ckks_hmult_relin_noalloc): CKKS_SCRATCH_BYTES of device memory per GPU,
// held for the life of the process.  Host code never passes the array's name
// to a kernel: its device address on each GPU is looked up once, with that
// GPU current, when a context is created there.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint64_t scratch[CKKS_SCRATCH_BYTES / 8];

namespace {

std::mutex g_scratch_mu;
std::map<int, u64 *> g_scratch_at;   // device -> address of its scratch array

u64 *scratch_address(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_at.find(dev);
    if (it != g_scratch_at.end()) return it->second;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        fail(CKKS_E_DEVICE, std::string("scratch array address: ") + hipGetErrorString(e));
    g_scratch_at[dev] = (u64 *)p;
    return (u64 *)p;
}

size_t round_words(size_t w) { return (w + 31) & ~(size_t)31; }

// scratch words the no-alloc product takes at level l for B ciphertexts:
// tensor (d01, d2) and accumulators for the whole call, then either the ModUp
// (its iNTT copy and the extended digits) or the ModDown (y, z) in one region
size_t hmult_scratch_words(ckks_ctx *c, int l, int B) {
    const size_t N = c->N;
    const int nq = l + 1, ne = nq + c->K;
    const int beta = (nq + c->alpha - 1) / c->alpha;
    size_t up = round_words((size_t)B * nq * N);
    for (int j = 0; j < beta; ++j) up += round_words((size_t)B * modup_table(c, l, j)->dout * N);
    const size_t down = round_words((size_t)2 * B * c->K * N) + round_words((size_t)2 * B * nq * N);
    return round_words((size_t)2 * B * nq * N) + round_words((size_t)B * nq * N) +
           round_words((size_t)2 * B * ne * N) + std::max(up, down);
}

// Mul_C and relinearisation of op_hmult (same kernels in the same order, so
// the same words) with every temporary carved from the GPU's scratch array;
// the result's words go to `out`, [B][2][l+1][N].
void hmult_noalloc(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, u64 *out, double *out_scale) {
    if (!c->have_keys) fail(CKKS_E_NOKEY, "no keys");
    if (a->level != b->level) fail(CKKS_E_LEVEL, "level mismatch");
    if (a->B != b->B) fail(CKKS_E_PARAM, "batch size mismatch");
    if (!c->scratch) fail(CKKS_E_DEVICE, "no scratch array on this device");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
        fail(CKKS_E_DEVICE, "the current device is not the context's");
    const int l = a->level, nq = l + 1, ne = nq + c->K, B = a->B;
    const size_t N = c->N;
    need_tables(c, l);
    const size_t need = hmult_scratch_words(c, l, B);
    if (need * 8 > (size_t)CKKS_SCRATCH_BYTES)
        fail(CKKS_E_PARAM, "this product needs " + std::to_string(need * 8) + " bytes of scratch, more than the " +
                               std::to_string((size_t)CKKS_SCRATCH_BYTES) + " bytes of CKKS_SCRATCH_BYTES");
    Carver cv{c->scratch, (size_t)CKKS_SCRATCH_BYTES / 8, 0};
    u64 *d01 = cv.take((size_t)B * 2 * nq * N), *d2 = cv.take((size_t)B * nq * N);
    u64 *acc = cv.take((size_t)B * 2 * ne * N);
    const size_t mark = cv.used;
    gpu::tensor(c->T, d01, d2, a->buf.p, b->buf.p, nq, B, map_q(0, nq), c->stream);
    ModUp mu;
    modup(c, l, d2, (size_t)nq * N, B, mu, &cv);
    gpu::InnerArgs ia = mu.ia;
    ia.key = c->relin.k.p;
    ia.perm = nullptr;
    gpu::key_inner(c->T, acc, ia, c->stream);
    // the ModUp's pieces are read only by the inner product, queued before
    // anything the ModDown writes over them (one stream)
    cv.used = mark;
    u64 *y = cv.take((size_t)2 * B * c->K * N), *z = cv.take((size_t)2 * B * nq * N);
    ks_moddown(c, l, B, acc, out, d01, 3, y, z);
    *out_scale = a->scale * b->scale;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

ckks_status ckks_ctx_create(const ckks_params *p, void *arena, size_t arena_bytes, void *hip_stream, ckks_ctx **out) {
    if (!p || !out) return CKKS_E_PARAM;
    *out = nullptr;
    const bool bts = p->bts_evalmod_levels > 0;
    const uint32_t Ltot = p->max_level + p->bts_stc_levels + p->bts_evalmod_levels + p->bts_cts_levels;
    if (p->log_n < 4 || p->log_n > 16 || p->max_level < 1 || p->num_special < 1 || p->digit_size < 1 ||
        Ltot + 1 + p->num_special > (uint32_t)gpu::kMaxLimbs || p->q0_bits > 61 || p->p_bits > 61 ||
        p->q0_bits < 30 || p->p_bits < 30 || p->log_scale < 20 || p->log_scale > 58 ||
        p->hamming_weight > (1u << p->log_n) || !(p->sigma > 0) ||
        (bts && (p->bts_stc_levels < 1 || p->bts_cts_levels < 1 || p->bts_log_scale < 20 || p->bts_log_scale > 60)) ||
        (!bts && (p->bts_stc_levels || p->bts_cts_levels)))
        return CKKS_E_PARAM;
    ckks_ctx *c = new ckks_ctx();
    ckks_status st = guard(c, [&] {
        c->prm = *p;
        c->logN = (int)p->log_n;
        c->N = 1 << c->logN;
        c->L = (int)Ltot;
        c->shape.l_after = (int)p->max_level;
        if (bts) {
            c->shape.n_stc = (int)p->bts_stc_levels;
            c->shape.n_evm = (int)p->bts_evalmod_levels;
            c->shape.n_cts = (int)p->bts_cts_levels;
            c->shape.bts_bits = (int)p->bts_log_scale;
        }
        c->K = (int)p->num_special;
        c->alpha = (int)p->digit_size;
        c->dnum = (c->L + 1 + c->alpha - 1) / c->alpha;
        if (c->dnum > gpu::kMaxDigits) fail(CKKS_E_PARAM, "too many digits");
        c->np = c->L + 1 + c->K;
        c->stream = (hipStream_t)hip_stream;
        c->pool.reset(new Pool(arena, arena_bytes));
        hm::prime_chain(c->logN, c->L, c->K, (int)p->log_scale, (int)p->q0_bits, (int)p->p_bits, c->shape, c->q,
                        c->ladder);
        c->cdt = hm::gaussian_table(p->sigma);
        {
            u64 qmax = 0;
            for (u64 v : c->q) qmax = std::max(qmax, v);
            const long double m = (long double)(qmax - 1);
            const long double t = std::ldexp(1.0L, 127) / (m * m);
            c->sum_terms = (int)std::min<long double>(gpu::kMaxSumTerms, std::floor(t));
            if (c->sum_terms < 1) fail(CKKS_E_PARAM, "primes too large for 128-bit accumulation");
        }
        build_tables(c);
        hipchk(hipGetDevice(&c->device), "current device");
        c->scratch = scratch_address(c->device);
    });
    if (st != CKKS_OK) {
        delete c;
        return st;
    }
    *out = c;
    return CKKS_OK;
}

void ckks_ctx_destroy(ckks_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

const char *ckks_last_error(const ckks_ctx *c) { return c ? c->err.c_str() : "null context"; }

ckks_status ckks_ctx_primes(const ckks_ctx *c, uint64_t *primes, double *ladder) {
    if (!c) return CKKS_E_PARAM;
    if (primes) std::memcpy(primes, c->q.data(), c->q.size() * 8);
    if (ladder) std::memcpy(ladder, c->ladder.data(), c->ladder.size() * 8);
    return CKKS_OK;
}

ckks_status ckks_set_stream(ckks_ctx *c, void *s) {
    if (!c) return CKKS_E_PARAM;
    c->stream = (hipStream_t)s;
    return CKKS_OK;
}

ckks_status ckks_mem_info(ckks_ctx *c, ckks_mem_stats *out, uint64_t *ct_bytes, int reset_peak) {
    if (!c || !out) return CKKS_E_PARAM;
    return guard(c, [&] {
        size_t fr = 0, tot = 0;
        hipchk(hipMemGetInfo(&fr, &tot), "device memory info");
        out->device_free = fr;
        out->device_total = tot;
        out->pool_cached = c->pool->cached();
        out->pool_in_use = c->pool->in_use();
        out->pool_peak = c->pool->peak();
        out->arena_left = c->pool->arena_left();
        if (ct_bytes)
            for (int l = 0; l <= c->L; ++l) ct_bytes[l] = c->words(l) * 8;
        if (reset_peak) c->pool->reset_peak();
    });
}

ckks_status ckks_stream_done(ckks_ctx *c, int *done) {
    if (!c || !done) return CKKS_E_PARAM;
    return guard(c, [&] {
        const hipError_t e = hipStreamQuery(c->stream);
        if (e == hipSuccess) *done = 1;
        else if (e == hipErrorNotReady) *done = 0;
        else hipchk(e, "stream query");
    });
}

ckks_status ckks_sync(ckks_ctx *c) {
    if (!c) return CKKS_E_PARAM;
    return guard(c, [&] { hipchk(hipStreamSynchronize(c->stream), "sync"); });
}

ckks_status ckks_keygen(ckks_ctx *c, uint64_t seed, const int32_t *galois, uint32_t n_galois) {
    if (!c || (n_galois && !galois)) return CKKS_E_PARAM;
    return guard(c, [&] { keygen(c, seed, galois, n_galois); });
}

int32_t ckks_galois_rotation(const ckks_ctx *c, int32_t steps) { return c ? galois_rot(c, steps) : 0; }

ckks_status ckks_encrypt(ckks_ctx *c, const double *x, uint32_t n, uint32_t level, double scale, uint64_t seed,
                         ckks_ct **out) {
    if (!c || (n && !x)) return CKKS_E_PARAM;
    return guard_out(c, out, [&] { return op_encrypt(c, x, n, (int)level, scale, seed); });
}

ckks_status ckks_encrypt_batch(ckks_ctx *c, const double *x, uint32_t n_ct, uint32_t n, uint32_t level, double scale,
                               uint64_t seed0, ckks_ct **outs) {
    if (!c || (n_ct && (!x || !outs))) return CKKS_E_PARAM;
    for (uint32_t i = 0; i < n_ct; ++i) outs[i] = nullptr;
    ckks_status st = guard(c, [&] {
        if (!c->have_keys) fail(CKKS_E_NOKEY, "no keys");
        if ((int)level > c->L) fail(CKKS_E_LEVEL, "bad level");
        if (n > (uint32_t)c->N / 2) fail(CKKS_E_PARAM, "too many slots");
        const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        const uint32_t chunk = 4 * hw;
        for (uint32_t off = 0; off < n_ct; off += chunk) {
            const uint32_t cnt = std::min(chunk, n_ct - off);
            std::vector<EncHost> hs(cnt);
            std::vector<std::thread> th;
            for (unsigned t = 0; t < hw; ++t)
                th.emplace_back([&, t] {
                    for (uint32_t i = t; i < cnt; i += hw)
                        enc_host(c, x + (size_t)(off + i) * n, n, scale, seed0 + off + i, hs[i]);
                });
            for (auto &t : th) t.join();
            for (uint32_t i = 0; i < cnt; ++i) {
                if (!hs[i].ok) fail(CKKS_E_RANGE, "value out of range for encoding");
                outs[off + i] = enc_device(c, hs[i], (int)level, scale).release();
            }
        }
    });
    if (st != CKKS_OK)
        for (uint32_t i = 0; i < n_ct; ++i) { delete outs[i]; outs[i] = nullptr; }
    return st;
}

ckks_status ckks_decrypt(ckks_ctx *c, const ckks_ct *ct, double *re, double *im) {
    if (!c || !ct || !re) return CKKS_E_PARAM;
    return guard(c, [&] { op_decrypt(c, ct, re, im); });
}

ckks_status ckks_ct_import(ckks_ctx *c, const uint64_t *host, uint32_t level, double scale, ckks_ct **out) {
    if (!c || !host) return CKKS_E_PARAM;
    return guard_out(c, out, [&] {
        if ((int)level > c->L) fail(CKKS_E_LEVEL, "bad level");
        Ct r = ct_new(c, (int)level, scale);
        hipchk(hipMemcpyAsync(r->buf.p, host, c->words(level) * 8, hipMemcpyHostToDevice, c->stream), "import");
        hipchk(hipStreamSynchronize(c->stream), "import sync");
        return r;
    });
}

ckks_status ckks_ct_export(ckks_ctx *c, const ckks_ct *ct, uint64_t *host) {
    if (!c || !ct || !host) return CKKS_E_PARAM;
    return guard(c, [&] {
        hipchk(hipMemcpyAsync(host, ct->buf.p, c->words(ct->level) * ct->B * 8, hipMemcpyDeviceToHost, c->stream),
               "export");
        hipchk(hipStreamSynchronize(c->stream), "export sync");
    });
}

void *ckks_ct_device_ptr(const ckks_ct *ct) { return ct ? (void *)ct->buf.p : nullptr; }
int32_t ckks_ct_level(const ckks_ct *ct) { return ct ? ct->level : -1; }
double ckks_ct_scale(const ckks_ct *ct) { return ct ? ct->scale : 0.0; }
void ckks_ct_free(ckks_ctx *c, ckks_ct *ct) {
    (void)c;
    delete ct;
}

#define CT_ARGS_CHECK(...)                         \
    if (!c || !a) return CKKS_E_PARAM;

ckks_status ckks_add(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, ckks_ct **out) {
    if (!c || !a || !b) return CKKS_E_PARAM;
    return guard_out(c, out, [&] { return op_addsub(c, a, b, false); });
}
ckks_status ckks_sub(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, ckks_ct **out) {
    if (!c || !a || !b) return CKKS_E_PARAM;
    return guard_out(c, out, [&] { return op_addsub(c, a, b, true); });
}
ckks_status ckks_mul_int(ckks_ctx *c, const ckks_ct *a, int64_t k, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_mul_int(c, a, k, a->scale); });
}
ckks_status ckks_mul_const(ckks_ctx *c, const ckks_ct *a, double v, double s_c, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_mul_const(c, a, v, s_c); });
}
ckks_status ckks_mul_const_down(ckks_ctx *c, const ckks_ct *a, double v, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_mul_const_down(c, a, v); });
}
ckks_status ckks_add_const(ckks_ctx *c, const ckks_ct *a, double v, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_add_const(c, a, v); });
}
ckks_status ckks_drop_level(ckks_ctx *c, const ckks_ct *a, uint32_t level, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_drop(c, a, (int)level); });
}
ckks_status ckks_level_to(ckks_ctx *c, const ckks_ct *a, uint32_t level, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_level_to(c, a, (int)level); });
}
ckks_status ckks_rescale(ckks_ctx *c, const ckks_ct *a, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_rescale(c, a); });
}
ckks_status ckks_hmult_relin(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, ckks_ct **out) {
    if (!c || !a || !b) return CKKS_E_PARAM;
    return guard_out(c, out, [&] { return op_hmult(c, a, b); });
}
ckks_status ckks_hmult_relin_noalloc(ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, uint64_t *out,
                                     double *out_scale) {
    if (!c || !a || !b || !out || !out_scale) return CKKS_E_PARAM;
    return guard(c, [&] { hmult_noalloc(c, a, b, out, out_scale); });
}
ckks_status ckks_rotate(ckks_ctx *c, const ckks_ct *a, int32_t steps, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_rotate(c, a, steps); });
}
ckks_status ckks_rotate_hoisted(ckks_ctx *c, const ckks_ct *a, const int32_t *steps, uint32_t n, ckks_ct **outs) {
    if (!c || !a || (n && (!steps || !outs))) return CKKS_E_PARAM;
    for (uint32_t i = 0; i < n; ++i) outs[i] = nullptr;
    return guard(c, [&] {
        std::vector<int> ks(steps, steps + n);
        std::vector<Ct> r = op_rotate_hoisted(c, a, ks);
        for (uint32_t i = 0; i < n; ++i) outs[i] = r[i].release();
    });
}
ckks_status ckks_conjugate(ckks_ctx *c, const ckks_ct *a, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_automorphism(c, a, 2 * c->N - 1); });
}
ckks_status ckks_cheb_eval(ckks_ctx *c, const ckks_ct *a, const double *coeffs, uint32_t degree, double lo,
                           double hi, ckks_ct **out) {
    if (!c || !a || !coeffs) return CKKS_E_PARAM;
    return guard_out(c, out, [&] {
        std::vector<double> cf(coeffs, coeffs + degree + 1);
        return op_cheb(c, a, cf, lo, hi);
    });
}
ckks_status ckks_cheb_coeffs_invsqrt(uint32_t degree, double a, double b, double *coeffs) {
    if (!coeffs || degree < 1 || !(a > 0) || !(b > a)) return CKKS_E_PARAM;
    hm::cheb_invsqrt((int)degree, a, b, coeffs);
    return CKKS_OK;
}
ckks_status ckks_newton_step(ckks_ctx *c, const ckks_ct *y, const ckks_ct *h, int raw_x, ckks_ct **out) {
    if (!c || !y || !h) return CKKS_E_PARAM;
    return guard_out(c, out, [&] { return op_newton(c, y, h, raw_x != 0); });
}
ckks_status ckks_bts_setup(ckks_ctx *c, double K, uint32_t r, uint32_t degree) {
    if (!c) return CKKS_E_PARAM;
    return guard(c, [&] { bts_setup(c, K, (int)r, (int)degree); });
}
ckks_status ckks_bts_rotations(const ckks_ctx *c, int32_t *steps, uint32_t cap, uint32_t *count) {
    if (!c || !count) return CKKS_E_PARAM;
    return guard(const_cast<ckks_ctx *>(c), [&] {
        std::vector<int> v = bts_rotations(c);
        *count = (uint32_t)v.size();
        for (uint32_t i = 0; i < cap && i < v.size(); ++i) steps[i] = v[i];
    });
}
ckks_status ckks_bootstrap(ckks_ctx *c, const ckks_ct *a, int64_t bound, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_bootstrap(c, a, bound); });
}
ckks_status ckks_mod_raise(ckks_ctx *c, const ckks_ct *a, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_mod_raise(c, a); });
}
ckks_status ckks_coeff_to_slot(ckks_ctx *c, const ckks_ct *a, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_coeff_to_slot(c, a); });
}
ckks_status ckks_eval_mod(ckks_ctx *c, const ckks_ct *a, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_eval_mod(c, a); });
}
ckks_status ckks_slot_to_coeff(ckks_ctx *c, const ckks_ct *a, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_slot_to_coeff(c, a); });
}
ckks_status ckks_mul_monomial(ckks_ctx *c, const ckks_ct *a, int32_t k, ckks_ct **out) {
    CT_ARGS_CHECK();
    return guard_out(c, out, [&] { return op_mul_monomial(c, a, k); });
}
static ckks_invsqrt_opts default_opts() {
    ckks_invsqrt_opts o;
    o.a = 0.0009765625;   // 2^-10
    o.b = 1.0;
    o.literal = 0;
    o.pre_bts = 0;
    o.bts_bound = 0;
    o.B = 0.0;
    return o;
}
ckks_status ckks_invsqrt(ckks_ctx *c, const ckks_ct *x, uint32_t degree, uint32_t iters, ckks_ct **out) {
    if (!c || !x) return CKKS_E_PARAM;
    ckks_invsqrt_opts o = default_opts();
    return guard_out(c, out, [&] { return op_invsqrt(c, x, (int)degree, (int)iters, o); });
}
ckks_status ckks_invsqrt_ex(ckks_ctx *c, const ckks_ct *x, uint32_t degree, uint32_t iters,
                            const ckks_invsqrt_opts *opts, ckks_ct **out) {
    if (!c || !x) return CKKS_E_PARAM;
    ckks_invsqrt_opts o = opts ? *opts : default_opts();
    return guard_out(c, out, [&] { return op_invsqrt(c, x, (int)degree, (int)iters, o); });
}
ckks_status ckks_invsqrt_batch(ckks_ctx *c, const ckks_ct *const *xs, uint32_t n, uint32_t degree, uint32_t iters,
                               const ckks_invsqrt_opts *opts, ckks_ct **outs) {
    if (!c || (n && (!xs || !outs))) return CKKS_E_PARAM;
    ckks_invsqrt_opts o = opts ? *opts : default_opts();
    for (uint32_t i = 0; i < n; ++i) outs[i] = nullptr;
    ckks_status st = guard(c, [&] {
        if (n == 0) return;
        for (uint32_t i = 0; i < n; ++i) {
            if (!xs[i] || xs[i]->B != 1) fail(CKKS_E_PARAM, "bad input ciphertext");
            if (xs[i]->level != xs[0]->level || xs[i]->scale != xs[0]->scale)
                fail(CKKS_E_PARAM, "batched inputs must share level and scale");
        }
        const size_t w = c->words(xs[0]->level);
        for (uint32_t off = 0; off < n; off += kMaxBatch) {
            const int B = (int)std::min<uint32_t>(kMaxBatch, n - off);
            Ct xb = ct_new(c, xs[0]->level, xs[0]->scale, B);
            for (int b = 0; b < B; ++b)
                hipchk(hipMemcpyAsync(xb->buf.p + (size_t)b * w, xs[off + b]->buf.p, w * 8, hipMemcpyDeviceToDevice,
                                      c->stream),
                       "gather");
            Ct yb = op_invsqrt(c, xb.get(), (int)degree, (int)iters, o);
            const size_t wy = c->words(yb->level);
            for (int b = 0; b < B; ++b) {
                Ct y1 = ct_new(c, yb->level, yb->scale, 1);
                hipchk(hipMemcpyAsync(y1->buf.p, yb->buf.p + (size_t)b * wy, wy * 8, hipMemcpyDeviceToDevice,
                                      c->stream),
                       "scatter");
                outs[off + b] = y1.release();
            }
        }
    });
    if (st != CKKS_OK)
        for (uint32_t i = 0; i < n; ++i) { delete outs[i]; outs[i] = nullptr; }
    return st;
}
ckks_status ckks_invsqrt_graph_create(ckks_ctx *c, const ckks_ct *x, uint32_t degree, uint32_t iters,
                                      const ckks_invsqrt_opts *opts, ckks_graph **out) {
    if (!c || !x || !out) return CKKS_E_PARAM;
    *out = nullptr;
    ckks_invsqrt_opts o = opts ? *opts : default_opts();
    return guard(c, [&] { *out = graph_create(c, x, (int)degree, (int)iters, o); });
}
ckks_status ckks_invsqrt_graph_run(ckks_ctx *c, ckks_graph *g, const ckks_ct *x, ckks_ct **out) {
    if (!c || !g || !x) return CKKS_E_PARAM;
    return guard_out(c, out, [&] { return graph_run(c, g, x); });
}
void ckks_graph_destroy(ckks_ctx *c, ckks_graph *g) {
    if (!c || !g) return;
    (void)hipStreamSynchronize(c->stream);
    graph_free(c, g);
}
ckks_status ckks_ct_pack(ckks_ctx *c, const ckks_ct *const *cts, uint32_t n, ckks_ct **out) {
    if (!c || !cts || n == 0) return CKKS_E_PARAM;
    return guard_out(c, out, [&] {
        for (uint32_t i = 0; i < n; ++i) {
            if (!cts[i] || cts[i]->B != 1) fail(CKKS_E_PARAM, "pack takes single ciphertexts");
            if (cts[i]->level != cts[0]->level || cts[i]->scale != cts[0]->scale)
                fail(CKKS_E_PARAM, "packed ciphertexts must share level and scale");
        }
        const size_t w = c->words(cts[0]->level);
        Ct r = ct_new(c, cts[0]->level, cts[0]->scale, (int)n);
        for (uint32_t i = 0; i < n; ++i)
            hipchk(hipMemcpyAsync(r->buf.p + i * w, cts[i]->buf.p, w * 8, hipMemcpyDeviceToDevice, c->stream), "pack");
        return r;
    });
}
ckks_status ckks_ct_unpack(ckks_ctx *c, const ckks_ct *batch, ckks_ct **outs) {
    if (!c || !batch || !outs) return CKKS_E_PARAM;
    for (int i = 0; i < batch->B; ++i) outs[i] = nullptr;
    ckks_status st = guard(c, [&] {
        const size_t w = c->words(batch->level);
        for (int i = 0; i < batch->B; ++i) {
            Ct r = ct_new(c, batch->level, batch->scale, 1);
            hipchk(hipMemcpyAsync(r->buf.p, batch->buf.p + i * w, w * 8, hipMemcpyDeviceToDevice, c->stream),
                   "unpack");
            outs[i] = r.release();
        }
    });
    if (st != CKKS_OK)
        for (int i = 0; i < batch->B; ++i) { delete outs[i]; outs[i] = nullptr; }
    return st;
}
int32_t ckks_ct_count(const ckks_ct *ct) { return ct ? ct->B : 0; }

ckks_status ckks_trace_enable(ckks_ctx *c, int on) {
    if (!c) return CKKS_E_PARAM;
    c->trace.clear();
    c->trace_on = on != 0;
    return CKKS_OK;
}
size_t ckks_trace_read(const ckks_ctx *c, char *buf, size_t cap) {
    if (!c) return 0;
    if (buf && cap) {
        size_t n = std::min(cap - 1, c->trace.size());
        std::memcpy(buf, c->trace.data(), n);
        buf[n] = 0;
    }
    return c->trace.size() + 1;
}

ckks_status ckks_ntt_device(ckks_ctx *c, uint64_t *data, uint32_t n_limbs, const uint32_t *prime_idx, int inverse) {
    if (!c || !data || !prime_idx || n_limbs == 0) return CKKS_E_PARAM;
    return guard(c, [&] {
        // launches take at most kMaxLimbs distinct limbs per map; chunk longer batches
        for (uint32_t off = 0; off < n_limbs; off += gpu::kMaxLimbs) {
            uint32_t cnt = std::min<uint32_t>(gpu::kMaxLimbs, n_limbs - off);
            LimbMap m{};
            for (uint32_t i = 0; i < cnt; ++i) {
                if (prime_idx[off + i] >= (uint32_t)c->np) fail(CKKS_E_PARAM, "bad prime index");
                m.p[i] = (uint8_t)prime_idx[off + i];
            }
            gpu::ntt(c->T, data + (size_t)off * c->N, (int)cnt, 1, m, inverse != 0, c->stream);
        }
    });
}

ckks_status ckks_ntt_schedule(ckks_ctx *c, int32_t r4_max_limbs, int32_t r8_max_limbs, int32_t s4_max_limbs) {
    if (!c || r4_max_limbs < -1 || r8_max_limbs < -1 || s4_max_limbs < -1) return CKKS_E_PARAM;
    return guard(c, [&] {
        c->T.ntt_r4_max = r4_max_limbs < 0 ? kNttR4Max : r4_max_limbs;
        c->T.ntt_r8_max = r8_max_limbs < 0 ? kNttR8Max : r8_max_limbs;
        c->T.ntt_s4_max = s4_max_limbs < 0 ? kNttS4Max : s4_max_limbs;
    });
}

ckks_status ckks_ntt_arith(ckks_ctx *c, int32_t fp64_max_bits) {
    if (!c || fp64_max_bits < -1 || fp64_max_bits > kNttFpBits) return CKKS_E_PARAM;
    return guard(c, [&] {
        c->T.fp_bits = c->logN != 16 ? 0 : fp64_max_bits < 0 ? kNttFpBits : fp64_max_bits;
    });
}

ckks_status ckks_butterfly_rate(ckks_ctx *c, int32_t form, uint64_t q, uint32_t rounds, uint32_t launches,
                                double *butterflies_per_s) {
    if (!c || !butterflies_per_s || form < 0 || form > 2 || rounds < 1 || rounds > 4096 || launches < 1 ||
        launches > 1000 || !(q & 1) || q < 3)
        return CKKS_E_PARAM;
    const uint64_t qmax = form == 0 ? (1ull << 61) : form == 1 ? (1ull << 42) : (1ull << 30);
    if (q >= qmax) return CKKS_E_PARAM;
    return guard(c, [&] {
        const size_t threads = (size_t)2048 * 256;   // 8 workgroups of 256 per compute unit
        const u64 w = (q / 3) | 1;                   // any residue: the rate does not depend on it
        const u64 wsh = form == 2 ? (u64)(((unsigned __int128)w << 32) / q)
                                  : (u64)(((unsigned __int128)w << 64) / q);
        const u64 inv64 = (u64)((((unsigned __int128)1) << 64) / q);
        const double wd = (double)w, wq = (double)w / (double)q, qinv = 1.0 / (double)q;
        Buf io(c->pool.get(), threads);
        std::vector<u64> h(threads);
        for (size_t i = 0; i < threads; ++i) h[i] = (i * 0x9e3779b97f4a7c15ull) >> 3;
        hipchk(hipMemcpyAsync(io.p, h.data(), threads * 8, hipMemcpyHostToDevice, c->stream), "copy");
        gpu::butterfly_rate(form, io.p, threads, (int)rounds, q, w, wsh, inv64, wd, wq, qinv, c->stream);   // warm-up
        hipEvent_t e0, e1;
        hipchk(hipEventCreate(&e0), "event");
        hipchk(hipEventCreate(&e1), "event");
        hipchk(hipEventRecord(e0, c->stream), "event");
        for (uint32_t k = 0; k < launches; ++k)
            gpu::butterfly_rate(form, io.p, threads, (int)rounds, q, w, wsh, inv64, wd, wq, qinv, c->stream);
        hipchk(hipEventRecord(e1, c->stream), "event");
        hipchk(hipEventSynchronize(e1), "sync");
        float ms = 0.f;
        hipchk(hipEventElapsedTime(&ms, e0, e1), "event");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *butterflies_per_s = (double)threads * rounds * 12.0 * launches / (ms * 1e-3);
    });
}

ckks_status ckks_profile_enable(ckks_ctx *c, int on) {
    if (!c) return CKKS_E_PARAM;
    return guard(c, [&] {
        hipchk(hipStreamSynchronize(c->stream), "sync");
        for (auto &f : c->prof)
            for (auto &e : f.second.ev) { c->ev_free.push_back(e.first); c->ev_free.push_back(e.second); }
        c->prof.clear();
        c->prof_on = on != 0;
    });
}
ckks_status ckks_profile_read(ckks_ctx *c, const char *family, uint64_t *calls, double *gpu_ms, double *alg_bytes) {
    if (!c || !family) return CKKS_E_PARAM;
    return guard(c, [&] {
        hipchk(hipStreamSynchronize(c->stream), "sync");
        double ms = 0;
        uint64_t n = 0;
        double by = 0;
        auto it = c->prof.find(family);
        if (it != c->prof.end()) {
            for (auto &e : it->second.ev) {
                float t = 0;
                hipchk(hipEventElapsedTime(&t, e.first, e.second), "elapsed");
                ms += t;
            }
            n = it->second.calls;
            by = it->second.bytes;
        }
        if (calls) *calls = n;
        if (gpu_ms) *gpu_ms = ms;
        if (alg_bytes) *alg_bytes = by;
    });
}

}  // extern "C"
