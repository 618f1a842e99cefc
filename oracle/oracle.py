"""ctypes front-end of the CPU oracle (test infrastructure only).

The oracle is a plain, slow, single-threaded C implementation of the RNS-CKKS
arithmetic and of the paper's CryptoInvSqrt (Alg. 1).  Only the test suite,
the smoke entry point and the CPU-baseline leg of the benchmark may import this
module; the GPU library never does.

Build: ``python -m oracle.build`` (or ``__graft_entry__.build()``) compiles
``liboracle.so`` next to this file with gcc.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB: another build of the same source (e.g. with sanitizers)
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

u64p = C.POINTER(C.c_uint64)
i64p = C.POINTER(C.c_int64)
dblp = C.POINTER(C.c_double)
i32p = C.POINTER(C.c_int32)
i8p = C.POINTER(C.c_int8)
vp = C.c_void_p


def _p(a, t):
    return a.ctypes.data_as(t)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise RuntimeError("oracle not built: run __graft_entry__.build()")
    L = C.CDLL(_LIB)
    sig = {
        "orc_last_error": (C.c_char_p, []),
        "orc_is_prime": (C.c_int, [C.c_uint64]),
        "orc_psi": (C.c_uint64, [C.c_uint64, C.c_int]),
        "orc_shake256": (None, [C.c_char_p, C.c_size_t, C.c_char_p, C.c_size_t]),
        "orc_ctx_create": (vp, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                C.c_int, C.c_int, C.c_int]),
        "orc_ctx_free": (None, [vp]),
        "orc_ctx_info": (C.c_int, [vp, u64p, dblp]),
        "orc_dnum": (C.c_int, [vp]),
        "orc_cdt": (C.c_int, [vp, u64p]),
        "orc_ntt": (None, [vp, C.c_int, u64p]),
        "orc_intt": (None, [vp, C.c_int, u64p]),
        "orc_keygen": (C.c_int, [vp, C.c_uint64, i32p, C.c_int]),
        "orc_secret": (C.c_int, [vp, i8p]),
        "orc_evk_export": (C.c_int, [vp, C.c_int, u64p]),
        "orc_pk_export": (C.c_int, [vp, u64p]),
        "orc_automorph_perm": (C.c_int, [vp, C.c_int, i32p]),
        "orc_dft_direct_test": (None, [C.c_int, dblp, dblp, dblp, dblp, C.c_int]),
        "orc_dft_fast_test": (None, [C.c_int, dblp, dblp, dblp, dblp, C.c_int]),
        "orc_encode": (C.c_int, [vp, dblp, dblp, C.c_int, C.c_double, i64p]),
        "orc_decode_coeffs": (C.c_int, [vp, i64p, C.c_double, dblp, dblp]),
        "orc_embed_direct": (C.c_int, [vp, i64p, dblp, dblp]),
        "orc_encrypt": (vp, [vp, dblp, C.c_int, C.c_int, C.c_double, C.c_uint64]),
        "orc_decrypt": (C.c_int, [vp, vp, dblp, dblp]),
        "orc_decrypt_coeffs": (C.c_int, [vp, vp, dblp]),
        "orc_ct_import": (vp, [vp, u64p, C.c_int, C.c_double]),
        "orc_ct_export": (C.c_int, [vp, vp, u64p]),
        "orc_ct_level": (C.c_int, [vp]),
        "orc_ct_scale": (C.c_double, [vp]),
        "orc_ct_free": (None, [vp]),
        "orc_add": (vp, [vp, vp, vp]),
        "orc_sub": (vp, [vp, vp, vp]),
        "orc_mul_int": (vp, [vp, vp, C.c_int64]),
        "orc_mul_const": (vp, [vp, vp, C.c_double, C.c_double]),
        "orc_mul_const_down": (vp, [vp, vp, C.c_double]),
        "orc_add_const": (vp, [vp, vp, C.c_double]),
        "orc_drop_level": (vp, [vp, vp, C.c_int]),
        "orc_rescale": (vp, [vp, vp]),
        "orc_level_to": (vp, [vp, vp, C.c_int]),
        "orc_keyswitch": (C.c_int, [vp, C.c_int, C.c_int, u64p, u64p, u64p]),
        "orc_hmult": (vp, [vp, vp, vp]),
        "orc_mult_rs": (vp, [vp, vp, vp]),
        "orc_automorphism": (vp, [vp, vp, C.c_int]),
        "orc_galois_rot": (C.c_int, [vp, C.c_int]),
        "orc_rotate": (vp, [vp, vp, C.c_int]),
        "orc_conjugate": (vp, [vp, vp]),
        "orc_cheb_coeffs_invsqrt": (C.c_int, [C.c_int, C.c_double, C.c_double, dblp]),
        "orc_cheb_coeffs_cosmod": (C.c_int, [C.c_int, C.c_double, C.c_double, dblp]),
        "orc_cheb_depth": (C.c_int, [C.c_int]),
        "orc_cheb_eval": (vp, [vp, vp, dblp, C.c_int, C.c_double, C.c_double]),
        "orc_newton_step": (vp, [vp, vp, vp]),
        "orc_newton_step_ex": (vp, [vp, vp, vp, C.c_int]),
        "orc_invsqrt": (vp, [vp, vp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int64, C.c_int,
                             C.c_double]),
        "orc_bootstrap": (vp, [vp, vp, C.c_int64]),
        "orc_ctx_create_bts": (vp, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.c_int, C.c_double, C.c_int, C.c_int, C.c_int]),
        "orc_bts_config": (C.c_int, [vp, C.c_double, C.c_int, C.c_int]),
        "orc_bts_rotations": (C.c_int, [vp, i32p, C.c_int]),
        "orc_mod_raise": (vp, [vp, vp]),
        "orc_mul_monomial": (vp, [vp, vp, C.c_int]),
        "orc_rotate_hoisted": (C.c_int, [vp, vp, i32p, C.c_int, C.POINTER(vp)]),
        "orc_coeff_to_slot": (vp, [vp, vp]),
        "orc_slot_to_coeff": (vp, [vp, vp]),
        "orc_eval_mod": (vp, [vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name, None)
        if f is None:
            continue
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class OracleError(RuntimeError):
    pass


def _chk(ptr):
    if not ptr:
        raise OracleError(lib().orc_last_error().decode())
    return ptr


class Ct:
    """Oracle ciphertext handle (host memory, NTT domain, [2][level+1][N])."""

    def __init__(self, ctx, ptr):
        self.ctx = ctx
        self.ptr = _chk(ptr)

    def __del__(self):
        try:
            if self.ptr:
                lib().orc_ct_free(self.ptr)
                self.ptr = None
        except Exception:
            pass

    @property
    def level(self):
        return lib().orc_ct_level(self.ptr)

    @property
    def scale(self):
        return lib().orc_ct_scale(self.ptr)

    def words(self):
        out = np.zeros((2, self.level + 1, self.ctx.N), dtype=np.uint64)
        lib().orc_ct_export(self.ctx.ptr, self.ptr, _p(out, u64p))
        return out


class Context:
    """Oracle parameter set + keys.  Arguments mirror the GPU library."""

    def __init__(self, logN, L, K, alpha, h=0, sigma=3.2, log_delta=40, q0_bits=60, p_bits=60, bts=None):
        """bts = (n_stc, n_evm, n_cts, bts_bits): a bootstrapping chain whose
        computation levels are 0..L and whose bootstrapping levels sit above."""
        self.N = 1 << logN
        self.n = self.N // 2
        if bts:
            n_stc, n_evm, n_cts, bts_bits = bts
            self.l_after = L
            ptr = lib().orc_ctx_create_bts(logN, L, n_stc, n_evm, n_cts, bts_bits, K, alpha, h, sigma,
                                           log_delta, q0_bits, p_bits)
            L = L + n_stc + n_evm + n_cts
        else:
            self.l_after = L
            ptr = lib().orc_ctx_create(logN, L, K, alpha, h, sigma, log_delta, q0_bits, p_bits)
        self.logN, self.L, self.K, self.alpha, self.h = logN, L, K, alpha, h
        self.ptr = _chk(ptr)
        self.np_ = L + 1 + K
        self.primes = np.zeros(self.np_, dtype=np.uint64)
        self.ladder = np.zeros(L + 1, dtype=np.float64)
        lib().orc_ctx_info(self.ptr, _p(self.primes, u64p), _p(self.ladder, dblp))
        self.dnum = lib().orc_dnum(self.ptr)
        self.galois = []

    @classmethod
    def from_set(cls, name, bootstrapping=True):
        """The named parameter set (the JSON data file of the library's
        package: numbers only, the primes are generated here) with its
        bootstrapping configured when it has one."""
        import json
        path = os.path.join(os.path.dirname(_HERE), "paper_2606_10477_amd", "params.json")
        with open(path) as f:
            s = json.load(f)[name]
        o = cls(s["log_n"], s["max_level"], s["num_special"], s["digit_size"], h=s["hamming_weight"],
                bts=tuple(s["bts"]) if "bts" in s else None)
        if bootstrapping and "evalmod" in s:
            e = s["evalmod"]
            o.bts_config(float(e["K"]), int(e["r"]), int(e["degree"]))
        return o

    def __del__(self):
        try:
            if self.ptr:
                lib().orc_ctx_free(self.ptr)
                self.ptr = None
        except Exception:
            pass

    # -- keys ------------------------------------------------------------
    def keygen(self, seed, galois=()):
        g = np.array(list(galois), dtype=np.int32)
        self.galois = list(galois)
        rc = lib().orc_keygen(self.ptr, seed, _p(g, i32p) if len(g) else None, len(g))
        if rc != 0:
            raise OracleError("keygen")

    def galois_rot(self, k):
        return lib().orc_galois_rot(self.ptr, k)

    def secret(self):
        s = np.zeros(self.N, dtype=np.int8)
        lib().orc_secret(self.ptr, _p(s, i8p))
        return s

    def evk(self, which=-1):
        out = np.zeros((self.dnum, 2, self.np_, self.N), dtype=np.uint64)
        lib().orc_evk_export(self.ptr, which, _p(out, u64p))
        return out

    def pk(self):
        out = np.zeros((2, self.L + 1, self.N), dtype=np.uint64)
        lib().orc_pk_export(self.ptr, _p(out, u64p))
        return out

    def cdt(self):
        out = np.zeros(64, dtype=np.uint64)
        k = lib().orc_cdt(self.ptr, _p(out, u64p))
        return out[:k]

    # -- transforms --------------------------------------------------------
    def ntt(self, pi, a):
        a = np.ascontiguousarray(a, dtype=np.uint64).copy()
        lib().orc_ntt(self.ptr, pi, _p(a, u64p))
        return a

    def intt(self, pi, a):
        a = np.ascontiguousarray(a, dtype=np.uint64).copy()
        lib().orc_intt(self.ptr, pi, _p(a, u64p))
        return a

    def automorph_perm(self, g):
        out = np.zeros(self.N, dtype=np.int32)
        lib().orc_automorph_perm(self.ptr, g, _p(out, i32p))
        return out

    def encode(self, re, im=None, scale=2.0 ** 40):
        re = np.ascontiguousarray(re, dtype=np.float64)
        im_ = None if im is None else np.ascontiguousarray(im, dtype=np.float64)
        out = np.zeros(self.N, dtype=np.int64)
        rc = lib().orc_encode(self.ptr, _p(re, dblp), None if im_ is None else _p(im_, dblp),
                              len(re), scale, _p(out, i64p))
        if rc != 0:
            raise OracleError("encode range")
        return out

    def decode_coeffs(self, m, scale):
        m = np.ascontiguousarray(m, dtype=np.int64)
        re = np.zeros(self.n)
        im = np.zeros(self.n)
        lib().orc_decode_coeffs(self.ptr, _p(m, i64p), scale, _p(re, dblp), _p(im, dblp))
        return re + 1j * im

    def embed_direct(self, m):
        m = np.ascontiguousarray(m, dtype=np.int64)
        re = np.zeros(self.n)
        im = np.zeros(self.n)
        lib().orc_embed_direct(self.ptr, _p(m, i64p), _p(re, dblp), _p(im, dblp))
        return re + 1j * im

    # -- ciphertexts -------------------------------------------------------
    def encrypt(self, x, level, scale, seed):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return Ct(self, lib().orc_encrypt(self.ptr, _p(x, dblp), len(x), level, scale, seed))

    def decrypt(self, ct):
        re = np.zeros(self.n)
        im = np.zeros(self.n)
        if lib().orc_decrypt(self.ptr, ct.ptr, _p(re, dblp), _p(im, dblp)) != 0:
            raise OracleError("decrypt")
        return re + 1j * im

    def decrypt_coeffs(self, ct):
        out = np.zeros(self.N)
        lib().orc_decrypt_coeffs(self.ptr, ct.ptr, _p(out, dblp))
        return out

    def ct_import(self, words, level, scale):
        w = np.ascontiguousarray(words, dtype=np.uint64)
        assert w.size == 2 * (level + 1) * self.N
        return Ct(self, lib().orc_ct_import(self.ptr, _p(w, u64p), level, scale))

    def add(self, a, b):
        return Ct(self, lib().orc_add(self.ptr, a.ptr, b.ptr))

    def sub(self, a, b):
        return Ct(self, lib().orc_sub(self.ptr, a.ptr, b.ptr))

    def mul_int(self, a, k):
        return Ct(self, lib().orc_mul_int(self.ptr, a.ptr, int(k)))

    def mul_const(self, a, v, s_c):
        return Ct(self, lib().orc_mul_const(self.ptr, a.ptr, float(v), float(s_c)))

    def mul_const_down(self, a, v):
        return Ct(self, lib().orc_mul_const_down(self.ptr, a.ptr, float(v)))

    def add_const(self, a, v):
        return Ct(self, lib().orc_add_const(self.ptr, a.ptr, float(v)))

    def drop_level(self, a, level):
        return Ct(self, lib().orc_drop_level(self.ptr, a.ptr, level))

    def rescale(self, a):
        return Ct(self, lib().orc_rescale(self.ptr, a.ptr))

    def level_to(self, a, level):
        return Ct(self, lib().orc_level_to(self.ptr, a.ptr, level))

    def keyswitch(self, which, level, d):
        d = np.ascontiguousarray(d, dtype=np.uint64)
        o0 = np.zeros_like(d)
        o1 = np.zeros_like(d)
        lib().orc_keyswitch(self.ptr, which, level, _p(d, u64p), _p(o0, u64p), _p(o1, u64p))
        return o0, o1

    def hmult(self, a, b):
        return Ct(self, lib().orc_hmult(self.ptr, a.ptr, b.ptr))

    def mult_rs(self, a, b):
        """Product, relinearisation and rescale in one ModDown (as the chains use)."""
        return Ct(self, lib().orc_mult_rs(self.ptr, a.ptr, b.ptr))

    def automorphism(self, a, g):
        return Ct(self, lib().orc_automorphism(self.ptr, a.ptr, g))

    def rotate(self, a, k):
        return Ct(self, lib().orc_rotate(self.ptr, a.ptr, k))

    def conjugate(self, a):
        return Ct(self, lib().orc_conjugate(self.ptr, a.ptr))

    def rotate_hoisted(self, a, steps):
        """Rotations of one ciphertext sharing one ModUp (hoisted)."""
        st = np.ascontiguousarray(steps, dtype=np.int32)
        outs = (vp * len(st))()
        if lib().orc_rotate_hoisted(self.ptr, a.ptr, _p(st, i32p), len(st), outs) != 0:
            raise OracleError(lib().orc_last_error().decode())
        return [Ct(self, outs[i]) for i in range(len(st))]

    def cheb_eval(self, x, coeffs, a, b):
        cf = np.ascontiguousarray(coeffs, dtype=np.float64)
        return Ct(self, lib().orc_cheb_eval(self.ptr, x.ptr, _p(cf, dblp), len(cf) - 1, a, b))

    def newton_step(self, y, cx, raw_x=False):
        return Ct(self, lib().orc_newton_step_ex(self.ptr, y.ptr, cx.ptr, int(raw_x)))

    def invsqrt(self, x, degree, iters, a, b, literal=False, bts_bound=0, pre_bts=False, B=0.0):
        return Ct(self, lib().orc_invsqrt(self.ptr, x.ptr, degree, iters, a, b, int(literal), int(bts_bound),
                                          int(pre_bts), float(B)))

    # -- bootstrapping -------------------------------------------------------
    def bts_config(self, K=25.0, r=4, degree=31):
        if lib().orc_bts_config(self.ptr, K, r, degree) != 0:
            raise OracleError(lib().orc_last_error().decode())

    def bts_rotations(self):
        k = lib().orc_bts_rotations(self.ptr, None, 0)
        if k < 0:
            raise OracleError(lib().orc_last_error().decode())
        out = np.zeros(k, dtype=np.int32)
        lib().orc_bts_rotations(self.ptr, _p(out, i32p), k)
        return [int(v) for v in out]

    def bts_galois(self):
        """Galois elements of the keys bootstrapping needs (rotations + conjugation)."""
        return [self.galois_rot(k) for k in self.bts_rotations()] + [2 * self.N - 1]

    def mod_raise(self, a):
        return Ct(self, lib().orc_mod_raise(self.ptr, a.ptr))

    def mul_monomial(self, a, k):
        return Ct(self, lib().orc_mul_monomial(self.ptr, a.ptr, k))

    def coeff_to_slot(self, a):
        return Ct(self, lib().orc_coeff_to_slot(self.ptr, a.ptr))

    def slot_to_coeff(self, a):
        return Ct(self, lib().orc_slot_to_coeff(self.ptr, a.ptr))

    def eval_mod(self, a):
        return Ct(self, lib().orc_eval_mod(self.ptr, a.ptr))

    def bootstrap(self, a, bound=1):
        """Bootstrap a ciphertext whose message is bounded by the integer `bound`."""
        return Ct(self, lib().orc_bootstrap(self.ptr, a.ptr, int(bound)))


def cheb_coeffs_invsqrt(d, a, b):
    out = np.zeros(d + 1)
    if lib().orc_cheb_coeffs_invsqrt(d, a, b, _p(out, dblp)) != 0:
        raise OracleError("cheb coeffs")
    return out


def cheb_depth(d):
    """Levels the oracle's Chebyshev evaluation of degree d consumes (on
    [-1, 1]; another interval adds the affine map's level)."""
    return int(lib().orc_cheb_depth(d))


def cheb_coeffs_cosmod(d, K, two_r):
    out = np.zeros(d + 1)
    lib().orc_cheb_coeffs_cosmod(d, K, two_r, _p(out, dblp))
    return out


def is_prime(n):
    return bool(lib().orc_is_prime(n))


def psi(q, N):
    return lib().orc_psi(q, N)


def shake256(data, n):
    out = C.create_string_buffer(n)
    lib().orc_shake256(data, len(data), out, n)
    return out.raw


def dft_fast(x, sign=1):
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    ore = np.zeros(len(x))
    oim = np.zeros(len(x))
    lib().orc_dft_fast_test(len(x), _p(re, dblp), _p(im, dblp), _p(ore, dblp), _p(oim, dblp), sign)
    return ore + 1j * oim


def dft_direct(x, sign=1):
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    ore = np.zeros(len(x))
    oim = np.zeros(len(x))
    lib().orc_dft_direct_test(len(x), _p(re, dblp), _p(im, dblp), _p(ore, dblp), _p(oim, dblp), sign)
    return ore + 1j * oim
