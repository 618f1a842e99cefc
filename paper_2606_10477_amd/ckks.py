"""Thin ctypes binding of libckks_hip.so (include/ckks.h).

Argument marshalling only: every homomorphic step runs in the HIP library.
PyTorch supplies the device memory arena and the stream.  Loading fails loudly
when the library has not been built; there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CKKS_LIB selects another build of this library (for comparing builds)
LIB_PATH = os.environ.get("CKKS_LIB") or os.path.join(_HERE, "libckks_hip.so")
_lib = None

vp = C.c_void_p
u64p = C.POINTER(C.c_uint64)
dblp = C.POINTER(C.c_double)
i32p = C.POINTER(C.c_int32)
u32p = C.POINTER(C.c_uint32)

STATUS = {0: "OK", -1: "E_PARAM", -2: "E_LEVEL", -3: "E_SCALE", -4: "E_NOKEY", -5: "E_OOM",
          -6: "E_DEVICE", -7: "E_RANGE"}


class Params(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("max_level", C.c_uint32), ("num_special", C.c_uint32),
                ("digit_size", C.c_uint32), ("hamming_weight", C.c_uint32), ("sigma", C.c_double),
                ("log_scale", C.c_uint32), ("q0_bits", C.c_uint32), ("p_bits", C.c_uint32),
                ("bts_stc_levels", C.c_uint32), ("bts_evalmod_levels", C.c_uint32),
                ("bts_cts_levels", C.c_uint32), ("bts_log_scale", C.c_uint32)]


class InvsqrtOpts(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("literal", C.c_int32), ("pre_bts", C.c_int32),
                ("bts_bound", C.c_int64), ("B", C.c_double)]


class MemStats(C.Structure):
    _fields_ = [("device_free", C.c_size_t), ("device_total", C.c_size_t), ("pool_cached", C.c_size_t),
                ("pool_in_use", C.c_size_t), ("pool_peak", C.c_size_t), ("arena_left", C.c_size_t)]


# name -> (restype, argtypes): every symbol of include/ckks.h
SIGNATURES = {
    "ckks_ctx_create": (C.c_int, [C.POINTER(Params), vp, C.c_size_t, vp, C.POINTER(vp)]),
    "ckks_ctx_destroy": (None, [vp]),
    "ckks_last_error": (C.c_char_p, [vp]),
    "ckks_ctx_primes": (C.c_int, [vp, u64p, dblp]),
    "ckks_set_stream": (C.c_int, [vp, vp]),
    "ckks_sync": (C.c_int, [vp]),
    "ckks_stream_done": (C.c_int, [vp, C.POINTER(C.c_int)]),
    "ckks_mem_info": (C.c_int, [vp, C.POINTER(MemStats), u64p, C.c_int]),
    "ckks_keygen": (C.c_int, [vp, C.c_uint64, i32p, C.c_uint32]),
    "ckks_galois_rotation": (C.c_int32, [vp, C.c_int32]),
    "ckks_encrypt": (C.c_int, [vp, dblp, C.c_uint32, C.c_uint32, C.c_double, C.c_uint64, C.POINTER(vp)]),
    "ckks_decrypt": (C.c_int, [vp, vp, dblp, dblp]),
    "ckks_encrypt_batch": (C.c_int, [vp, dblp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_double, C.c_uint64,
                                     C.POINTER(vp)]),
    "ckks_ct_import": (C.c_int, [vp, u64p, C.c_uint32, C.c_double, C.POINTER(vp)]),
    "ckks_ct_export": (C.c_int, [vp, vp, u64p]),
    "ckks_ct_device_ptr": (vp, [vp]),
    "ckks_ct_level": (C.c_int32, [vp]),
    "ckks_ct_scale": (C.c_double, [vp]),
    "ckks_ct_free": (None, [vp, vp]),
    "ckks_add": (C.c_int, [vp, vp, vp, C.POINTER(vp)]),
    "ckks_sub": (C.c_int, [vp, vp, vp, C.POINTER(vp)]),
    "ckks_mul_int": (C.c_int, [vp, vp, C.c_int64, C.POINTER(vp)]),
    "ckks_mul_const": (C.c_int, [vp, vp, C.c_double, C.c_double, C.POINTER(vp)]),
    "ckks_mul_const_down": (C.c_int, [vp, vp, C.c_double, C.POINTER(vp)]),
    "ckks_add_const": (C.c_int, [vp, vp, C.c_double, C.POINTER(vp)]),
    "ckks_drop_level": (C.c_int, [vp, vp, C.c_uint32, C.POINTER(vp)]),
    "ckks_level_to": (C.c_int, [vp, vp, C.c_uint32, C.POINTER(vp)]),
    "ckks_rescale": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckks_hmult_relin": (C.c_int, [vp, vp, vp, C.POINTER(vp)]),
    "ckks_hmult_relin_noalloc": (C.c_int, [vp, vp, vp, vp, dblp]),
    "ckks_rotate": (C.c_int, [vp, vp, C.c_int32, C.POINTER(vp)]),
    "ckks_conjugate": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckks_rotate_hoisted": (C.c_int, [vp, vp, i32p, C.c_uint32, C.POINTER(vp)]),
    "ckks_cheb_eval": (C.c_int, [vp, vp, dblp, C.c_uint32, C.c_double, C.c_double, C.POINTER(vp)]),
    "ckks_cheb_coeffs_invsqrt": (C.c_int, [C.c_uint32, C.c_double, C.c_double, dblp]),
    "ckks_newton_step": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(vp)]),
    "ckks_bootstrap": (C.c_int, [vp, vp, C.c_int64, C.POINTER(vp)]),
    "ckks_bts_setup": (C.c_int, [vp, C.c_double, C.c_uint32, C.c_uint32]),
    "ckks_bts_rotations": (C.c_int, [vp, i32p, C.c_uint32, u32p]),
    "ckks_mod_raise": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckks_coeff_to_slot": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckks_eval_mod": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckks_slot_to_coeff": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckks_mul_monomial": (C.c_int, [vp, vp, C.c_int32, C.POINTER(vp)]),
    "ckks_invsqrt": (C.c_int, [vp, vp, C.c_uint32, C.c_uint32, C.POINTER(vp)]),
    "ckks_invsqrt_ex": (C.c_int, [vp, vp, C.c_uint32, C.c_uint32, C.POINTER(InvsqrtOpts), C.POINTER(vp)]),
    "ckks_invsqrt_batch": (C.c_int, [vp, C.POINTER(vp), C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.POINTER(InvsqrtOpts), C.POINTER(vp)]),
    "ckks_ntt_device": (C.c_int, [vp, C.c_void_p, C.c_uint32, u32p, C.c_int]),
    "ckks_ntt_schedule": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32]),
    "ckks_ntt_arith": (C.c_int, [vp, C.c_int32]),
    "ckks_butterfly_rate": (C.c_int, [vp, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32, dblp]),
    "ckks_invsqrt_graph_create": (C.c_int, [vp, vp, C.c_uint32, C.c_uint32, C.POINTER(InvsqrtOpts),
                                            C.POINTER(vp)]),
    "ckks_invsqrt_graph_run": (C.c_int, [vp, vp, vp, C.POINTER(vp)]),
    "ckks_graph_destroy": (None, [vp, vp]),
    "ckks_ct_pack": (C.c_int, [vp, C.POINTER(vp), C.c_uint32, C.POINTER(vp)]),
    "ckks_ct_unpack": (C.c_int, [vp, vp, C.POINTER(vp)]),
    "ckks_ct_count": (C.c_int32, [vp]),
    "ckks_profile_enable": (C.c_int, [vp, C.c_int]),
    "ckks_trace_enable": (C.c_int, [vp, C.c_int]),
    "ckks_trace_read": (C.c_size_t, [vp, C.c_char_p, C.c_size_t]),
    "ckks_profile_read": (C.c_int, [vp, C.c_char_p, u64p, dblp, dblp]),
}


def library_sha256():
    """SHA-256 of the built library file (what a tuning table was measured with)."""
    import hashlib
    with open(LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libckks_hip.so is not built (run __graft_entry__.build()); "
                           "there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class CkksError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _p(a, t):
    return a.ctypes.data_as(t)


class Ciphertext:
    def __init__(self, ctx, ptr):
        self.ctx = ctx
        self.ptr = ptr

    def __del__(self):
        self.free()

    def free(self):
        try:
            if getattr(self, "ptr", None) and self.ctx.ptr:
                lib().ckks_ct_free(self.ctx.ptr, self.ptr)
        except TypeError:      # interpreter shutdown: the module's globals are gone
            pass
        self.ptr = None

    @property
    def level(self):
        return lib().ckks_ct_level(self.ptr)

    @property
    def scale(self):
        return lib().ckks_ct_scale(self.ptr)

    @property
    def count(self):
        return lib().ckks_ct_count(self.ptr)

    def words(self):
        B = self.count
        shape = (2, self.level + 1, self.ctx.N) if B == 1 else (B, 2, self.level + 1, self.ctx.N)
        out = np.zeros(shape, dtype=np.uint64)
        self.ctx._chk(lib().ckks_ct_export(self.ctx.ptr, self.ptr, _p(out, u64p)))
        return out


class InvsqrtGraph:
    """A captured CryptoInvSqrt chain (see ckks_invsqrt_graph_create)."""

    def __init__(self, ctx, ptr):
        self.ctx = ctx
        self.ptr = ptr

    def run(self, x):
        return self.ctx._ct(lib().ckks_invsqrt_graph_run, self.ptr, x.ptr)

    def close(self):
        try:
            if self.ptr and self.ctx.ptr:
                lib().ckks_graph_destroy(self.ctx.ptr, self.ptr)
        except TypeError:      # interpreter shutdown
            pass
        self.ptr = None

    def __del__(self):
        self.close()


class Context:
    """A parameter set on the current GPU.  `arena_bytes` > 0 allocates the
    context's device memory as one torch tensor (PyTorch owns the memory); the
    current torch stream orders all work."""

    def __init__(self, log_n, max_level, num_special, digit_size, hamming_weight=0, sigma=3.2,
                 log_scale=40, q0_bits=60, p_bits=60, arena_bytes=0, stream=None, bts=None):
        """bts = (stc_levels, evalmod_levels, cts_levels, bts_log_scale): a
        bootstrapping chain whose computation levels are 0..max_level
        (l_afterBTS) with the bootstrapping levels above."""
        import torch
        self.N = 1 << log_n
        self.n = self.N // 2
        bl = tuple(bts) if bts else (0, 0, 0, 0)
        self.l_after = max_level
        self.L = max_level + bl[0] + bl[1] + bl[2]
        self.K = num_special
        self.np_ = self.L + 1 + num_special
        p = Params(log_n, max_level, num_special, digit_size, hamming_weight, sigma, log_scale, q0_bits, p_bits,
                   *bl)
        self._arena = None
        arena_ptr = None
        if arena_bytes:
            self._arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
            arena_ptr = self._arena.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        out = vp()
        self.ptr = None
        st = lib().ckks_ctx_create(C.byref(p), arena_ptr, arena_bytes, stream, C.byref(out))
        if st != 0:
            raise CkksError(st, "context creation failed")
        self.ptr = out.value
        self.primes = np.zeros(self.np_, dtype=np.uint64)
        self.ladder = np.zeros(self.L + 1)
        lib().ckks_ctx_primes(self.ptr, _p(self.primes, u64p), _p(self.ladder, dblp))

    @classmethod
    def from_set(cls, name, bootstrapping=True, **kw):
        """A context on the named parameter set of params.json; on a
        bootstrapping set its EvalMod is configured too (bootstrapping=True).
        Keys still come from keygen."""
        from . import params
        ctx = cls(**params.context_kwargs(name), **kw)
        ev = params.evalmod(name)
        if bootstrapping and ev is not None:
            ctx.bts_setup(*ev)
        return ctx

    def close(self):
        if self.ptr:
            lib().ckks_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != 0:
            raise CkksError(st, lib().ckks_last_error(self.ptr).decode())

    def _ct(self, fn, *args):
        out = vp()
        self._chk(fn(self.ptr, *args, C.byref(out)))
        return Ciphertext(self, out.value)

    def sync(self):
        self._chk(lib().ckks_sync(self.ptr))

    def stream_done(self):
        """True when every operation queued on the context's stream has finished."""
        d = C.c_int()
        self._chk(lib().ckks_stream_done(self.ptr, C.byref(d)))
        return bool(d.value)

    def mem_info(self, reset_peak=False):
        """ckks_mem_info as a dict (bytes), with "ct_bytes" per level."""
        st = MemStats()
        cb = np.zeros(self.L + 1, dtype=np.uint64)
        self._chk(lib().ckks_mem_info(self.ptr, C.byref(st), _p(cb, u64p), int(reset_peak)))
        d = {k: int(getattr(st, k)) for k, _ in MemStats._fields_}
        d["ct_bytes"] = [int(v) for v in cb]
        return d

    def keygen(self, seed, galois=()):
        g = np.array(list(galois), dtype=np.int32)
        self._chk(lib().ckks_keygen(self.ptr, seed, _p(g, i32p) if len(g) else None, len(g)))

    def galois_rot(self, k):
        return lib().ckks_galois_rotation(self.ptr, k)

    def encrypt(self, x, level, scale, seed):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return self._ct(lib().ckks_encrypt, _p(x, dblp), len(x), level, scale, seed)

    def encrypt_batch(self, X, level, scale, seed0):
        X = np.ascontiguousarray(X, dtype=np.float64)
        n_ct, n = X.shape
        outs = (vp * n_ct)()
        self._chk(lib().ckks_encrypt_batch(self.ptr, _p(X, dblp), n_ct, n, level, scale, seed0, outs))
        return [Ciphertext(self, outs[i]) for i in range(n_ct)]

    def decrypt(self, ct):
        re = np.zeros(self.n)
        im = np.zeros(self.n)
        self._chk(lib().ckks_decrypt(self.ptr, ct.ptr, _p(re, dblp), _p(im, dblp)))
        return re + 1j * im

    def ct_import(self, words, level, scale):
        w = np.ascontiguousarray(words, dtype=np.uint64)
        assert w.size == 2 * (level + 1) * self.N
        return self._ct(lib().ckks_ct_import, _p(w, u64p), level, scale)

    def add(self, a, b):
        return self._ct(lib().ckks_add, a.ptr, b.ptr)

    def sub(self, a, b):
        return self._ct(lib().ckks_sub, a.ptr, b.ptr)

    def mul_int(self, a, k):
        return self._ct(lib().ckks_mul_int, a.ptr, int(k))

    def mul_const(self, a, v, s_c):
        return self._ct(lib().ckks_mul_const, a.ptr, float(v), float(s_c))

    def mul_const_down(self, a, v):
        return self._ct(lib().ckks_mul_const_down, a.ptr, float(v))

    def add_const(self, a, v):
        return self._ct(lib().ckks_add_const, a.ptr, float(v))

    def drop_level(self, a, level):
        return self._ct(lib().ckks_drop_level, a.ptr, level)

    def level_to(self, a, level):
        return self._ct(lib().ckks_level_to, a.ptr, level)

    def rescale(self, a):
        return self._ct(lib().ckks_rescale, a.ptr)

    def hmult(self, a, b):
        return self._ct(lib().ckks_hmult_relin, a.ptr, b.ptr)

    def hmult_noalloc(self, a, b, out_ptr):
        """ckks_hmult_relin_noalloc: the product's words into the device memory
        at out_ptr ([B][2][level+1][N] uint64, caller-owned); returns the scale."""
        sc = C.c_double()
        self._chk(lib().ckks_hmult_relin_noalloc(self.ptr, a.ptr, b.ptr, C.c_void_p(out_ptr), C.byref(sc)))
        return sc.value

    def rotate(self, a, k):
        return self._ct(lib().ckks_rotate, a.ptr, k)

    def conjugate(self, a):
        return self._ct(lib().ckks_conjugate, a.ptr)

    def cheb_eval(self, x, coeffs, a, b):
        cf = np.ascontiguousarray(coeffs, dtype=np.float64)
        return self._ct(lib().ckks_cheb_eval, x.ptr, _p(cf, dblp), len(cf) - 1, a, b)

    def newton_step(self, y, half_x, raw_x=False):
        return self._ct(lib().ckks_newton_step, y.ptr, half_x.ptr, int(raw_x))

    def rotate_hoisted(self, a, steps):
        st = np.ascontiguousarray(steps, dtype=np.int32)
        outs = (vp * len(st))()
        self._chk(lib().ckks_rotate_hoisted(self.ptr, a.ptr, _p(st, i32p), len(st), outs))
        return [Ciphertext(self, outs[i]) for i in range(len(st))]

    # -- bootstrapping -------------------------------------------------------
    def bts_setup(self, K=25.0, r=4, degree=31):
        self._chk(lib().ckks_bts_setup(self.ptr, K, r, degree))

    def bts_rotations(self):
        cnt = C.c_uint32()
        self._chk(lib().ckks_bts_rotations(self.ptr, None, 0, C.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.int32)
        self._chk(lib().ckks_bts_rotations(self.ptr, _p(out, i32p), cnt.value, C.byref(cnt)))
        return [int(v) for v in out]

    def bts_galois(self):
        """Galois elements of the keys bootstrapping needs (rotations + conjugation)."""
        return [self.galois_rot(k) for k in self.bts_rotations()] + [2 * self.N - 1]

    def bootstrap(self, a, bound=1):
        return self._ct(lib().ckks_bootstrap, a.ptr, int(bound))

    def mod_raise(self, a):
        return self._ct(lib().ckks_mod_raise, a.ptr)

    def coeff_to_slot(self, a):
        return self._ct(lib().ckks_coeff_to_slot, a.ptr)

    def eval_mod(self, a):
        return self._ct(lib().ckks_eval_mod, a.ptr)

    def slot_to_coeff(self, a):
        return self._ct(lib().ckks_slot_to_coeff, a.ptr)

    def mul_monomial(self, a, k):
        return self._ct(lib().ckks_mul_monomial, a.ptr, int(k))

    def invsqrt(self, x, degree, iters, a=2.0 ** -10, b=1.0, literal=False, bts_bound=0, pre_bts=False, B=0.0):
        o = InvsqrtOpts(a, b, int(literal), int(pre_bts), int(bts_bound), float(B))
        return self._ct(lib().ckks_invsqrt_ex, x.ptr, degree, iters, C.byref(o))

    def invsqrt_batch(self, xs, degree, iters, a=2.0 ** -10, b=1.0, literal=False, bts_bound=0, pre_bts=False,
                      B=0.0):
        o = InvsqrtOpts(a, b, int(literal), int(pre_bts), int(bts_bound), float(B))
        arr = (vp * len(xs))(*[x.ptr for x in xs])
        outs = (vp * len(xs))()
        self._chk(lib().ckks_invsqrt_batch(self.ptr, arr, len(xs), degree, iters, C.byref(o), outs))
        return [Ciphertext(self, outs[i]) for i in range(len(xs))]

    def profile(self, on=True):
        self._chk(lib().ckks_profile_enable(self.ptr, int(on)))

    def trace(self, on=True):
        self._chk(lib().ckks_trace_enable(self.ptr, int(on)))

    def trace_read(self):
        n = lib().ckks_trace_read(self.ptr, None, 0)
        buf = C.create_string_buffer(n)
        lib().ckks_trace_read(self.ptr, buf, n)
        out = []
        for line in buf.value.decode().splitlines():
            op, lvl, B = line.split()
            out.append((op, int(lvl), int(B)))
        return out

    def profile_read(self, family):
        n = C.c_uint64()
        ms = C.c_double()
        by = C.c_double()
        self._chk(lib().ckks_profile_read(self.ptr, family.encode(), C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def invsqrt_graph(self, x, degree, iters, a=2.0 ** -10, b=1.0, literal=False, bts_bound=0, pre_bts=False,
                      B=0.0):
        """Capture the chain for inputs shaped like x (level, scale, batch);
        returns an InvsqrtGraph whose run(x) replays it."""
        o = InvsqrtOpts(a, b, int(literal), int(pre_bts), int(bts_bound), float(B))
        out = vp()
        self._chk(lib().ckks_invsqrt_graph_create(self.ptr, x.ptr, degree, iters, C.byref(o), C.byref(out)))
        return InvsqrtGraph(self, out.value)

    def pack(self, cts):
        arr = (vp * len(cts))(*[x.ptr for x in cts])
        return self._ct(lib().ckks_ct_pack, arr, len(cts))

    def unpack(self, batch):
        B = batch.count
        outs = (vp * B)()
        self._chk(lib().ckks_ct_unpack(self.ptr, batch.ptr, outs))
        return [Ciphertext(self, outs[i]) for i in range(B)]

    def ntt_schedule(self, r4_max_limbs, r8_max_limbs, s4_max_limbs=-1):
        """Words per thread (and, for 4 words, sub-transforms per workgroup)
        of the N = 2^16 transforms by call size."""
        self._chk(lib().ckks_ntt_schedule(self.ptr, int(r4_max_limbs), int(r8_max_limbs), int(s4_max_limbs)))

    def ntt_arith(self, fp64_max_bits):
        """Primes below 2^fp64_max_bits transform in binary64 (0: none, -1: default)."""
        self._chk(lib().ckks_ntt_arith(self.ptr, int(fp64_max_bits)))

    def butterfly_rate(self, form, q, rounds=128, launches=20):
        """Forward NTT butterflies per second in registers (a word-size
        measurement): form 0 = 64-bit words (q < 2^61), 1 = binary64
        (q < 2^42), 2 = 32-bit words (q < 2^30)."""
        r = C.c_double()
        self._chk(lib().ckks_butterfly_rate(self.ptr, int(form), int(q), int(rounds), int(launches), C.byref(r)))
        return r.value

    def ntt_device(self, ptr, n_limbs, prime_idx, inverse=False):
        pi = np.ascontiguousarray(prime_idx, dtype=np.uint32)
        self._chk(lib().ckks_ntt_device(self.ptr, ptr, n_limbs, _p(pi, u32p), int(inverse)))


def cheb_coeffs_invsqrt(degree, a, b):
    out = np.zeros(degree + 1)
    st = lib().ckks_cheb_coeffs_invsqrt(degree, a, b, _p(out, dblp))
    if st != 0:
        raise CkksError(st, "bad arguments")
    return out
