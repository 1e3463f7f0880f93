"""ctypes wrapper of the C oracle (test infrastructure; see oracle/__init__.py).

Ciphertexts are coefficient-domain arrays of shape (2, level+1, N) with
canonical residues in [0, q_i), the format the GPU library exports for parity.
"""
import ctypes as C
import os

import numpy as np

from .build import build_oracle, oracle_lib_path

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ORACLE_LIB selects another build of the same source (the sanitizer test)
    path = os.environ.get("ORACLE_LIB") or oracle_lib_path()
    if not os.path.exists(path):
        build_oracle()
    lib = C.CDLL(path)
    vp, u64, i64, dbl, ci = C.c_void_p, C.c_uint64, C.c_int64, C.c_double, C.c_int
    P = C.POINTER
    sig = {
        "orc_create": (vp, [ci, ci, ci, ci, ci, ci, ci, ci, ci, ci]),
        "orc_destroy": (None, [vp]),
        "orc_num_primes": (ci, [vp]),
        "orc_primes": (None, [vp, P(u64)]),
        "orc_psi": (u64, [vp, ci]),
        "orc_counters": (None, [vp, P(i64)]),
        "orc_reset_counters": (None, [vp]),
        "orc_set_textbook": (None, [vp, ci]),
        "orc_ring_mul": (None, [vp, ci, P(u64), P(u64), P(u64)]),
        "orc_ntt_roundtrip": (None, [vp, ci, P(u64)]),
        "orc_ct_import": (vp, [vp, P(u64), ci, dbl]),
        "orc_ct_export": (None, [vp, vp, P(u64)]),
        "orc_ct_level": (ci, [vp]),
        "orc_ct_scale": (dbl, [vp]),
        "orc_ct_free": (None, [vp]),
        "orc_encode": (None, [vp, P(dbl), ci, dbl, P(i64)]),
        "orc_decode": (None, [vp, P(i64), dbl, ci, P(dbl)]),
        "orc_gen_secret": (None, [vp, u64]),
        "orc_get_secret": (None, [vp, P(i64)]),
        "orc_keygen": (None, [vp, u64, P(i64), ci]),
        "orc_get_key": (ci, [vp, u64, ci, ci, ci, P(u64)]),
        "orc_encrypt": (vp, [vp, P(i64), dbl, u64]),
        "orc_decrypt": (None, [vp, vp, P(i64)]),
        "orc_decrypt_decode": (None, [vp, vp, ci, P(dbl)]),
        "orc_add": (vp, [vp, vp, vp]),
        "orc_sub": (vp, [vp, vp, vp]),
        "orc_add_const": (vp, [vp, vp, dbl]),
        "orc_rescale": (vp, [vp, vp]),
        "orc_lower": (vp, [vp, vp, ci]),
        "orc_mul_const": (vp, [vp, vp, dbl, dbl]),
        "orc_mul_plain": (vp, [vp, vp, P(dbl), ci, dbl]),
        "orc_mul_relin": (vp, [vp, vp, vp]),
        "orc_mul_relin_rescale": (vp, [vp, vp, vp]),
        "orc_rotate": (vp, [vp, vp, i64]),
        "orc_rotate_hoisted": (None, [vp, vp, P(i64), ci, P(vp)]),
        "orc_refresh": (vp, [vp, vp, u64, u64]),
        "orc_key_switch": (None, [vp, u64, P(u64), ci, P(u64), P(u64)]),
        "orc_key_switch_raw": (None, [vp, u64, P(u64), ci, P(u64), P(u64)]),
        "orc_relin_rescale3": (vp, [vp, P(u64), ci, dbl]),
        "orc_lincomb": (vp, [vp, vp, dbl, vp, dbl, dbl, ci]),
        "orc_automorph": (None, [vp, ci, P(u64), u64, P(u64)]),
        "orc_galois_elt": (u64, [vp, i64]),
        "orc_sign_coeffs": (None, [P(dbl), P(dbl)]),
        "orc_eval_odd9": (vp, [vp, vp, P(dbl), dbl, dbl]),
        "orc_layout": (None, [vp, P(dbl), ci, ci, P(dbl)]),
        "orc_encrypt_logits": (vp, [vp, P(dbl), ci, ci, u64]),
        "orc_eval_argmax": (vp, [vp, vp, ci, ci, dbl, dbl, u64]),
        "orc_eval_argmax_phoenix": (vp, [vp, vp, ci, ci, dbl, dbl, u64]),
        "orc_packed_shape": (ci, [vp, ci, P(ci), P(ci), P(ci)]),
        "orc_layout_packed": (None, [vp, ci, P(dbl), P(ci), P(ci), P(dbl)]),
        "orc_encrypt_packed": (vp, [vp, ci, P(dbl), P(ci), P(ci), u64]),
        "orc_eval_argmax_packed": (vp, [vp, vp, ci, P(ci), P(ci), P(dbl), P(dbl), u64]),
        "orc_encode_complex": (None, [vp, P(dbl), P(dbl), ci, dbl, P(i64)]),
        "orc_set_boot": (ci, [vp, ci, ci, ci, ci, ci, ci, ci]),
        "orc_boot_steps": (ci, [vp, P(i64), ci]),
        "orc_boot_cheb": (None, [vp, P(dbl)]),
        "orc_boot_out_level": (ci, [vp]),
        "orc_boot_group_apply": (None, [vp, ci, ci, P(dbl), P(dbl), P(dbl), P(dbl)]),
        "orc_mod_raise": (vp, [vp, vp]),
        "orc_mul_monomial_half": (vp, [vp, vp, ci]),
        "orc_eval_mod": (vp, [vp, vp]),
        "orc_bootstrap": (vp, [vp, vp]),
        "orc_bootstrap_sparse": (vp, [vp, vp]),
        "orc_bootstrap_packed": (None, [vp, P(vp), ci, P(vp)]),
        "orc_set_boot_sparse": (ci, [vp, ci]),
        "orc_boot_sparse_apply": (None, [vp, ci, P(dbl), P(dbl), P(dbl), P(dbl)]),
        "orc_boot_transform_sparse": (vp, [vp, vp, ci]),
        "orc_boot_transform": (vp, [vp, vp, ci]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


def sign_coeffs():
    """(f, g) odd coefficients c1, c3, c5, c7, c9 of the two degree-9 polynomials."""
    lib = _load()
    f = np.zeros(5)
    g = np.zeros(5)
    lib.orc_sign_coeffs(_p(f, C.c_double), _p(g, C.c_double))
    return f, g


class Ct:
    """Oracle ciphertext handle."""

    def __init__(self, orc, handle):
        self._orc = orc
        self.h = handle

    def __del__(self):
        if self.h and _lib is not None:
            _lib.orc_ct_free(self.h)
            self.h = None

    @property
    def level(self):
        return _lib.orc_ct_level(self.h)

    @property
    def scale(self):
        return _lib.orc_ct_scale(self.h)

    def export(self):
        n = self._orc.n
        out = np.zeros((2, self.level + 1, n), dtype=np.uint64)
        _lib.orc_ct_export(self._orc.h, self.h, _p(out, C.c_uint64))
        return out


class Oracle:
    """Plain RNS-CKKS context: chain primes q_0..q_L, special primes p_0..p_{alpha-1}."""

    def __init__(self, log_n, n_q, q_bits, n_p, p_bits, log_scale, dg=2, df=2, min_level=1, refresh_level=0):
        self.lib = _load()
        self.h = self.lib.orc_create(log_n, n_q, q_bits, n_p, p_bits, log_scale, dg, df, min_level, refresh_level)
        self.refresh_level = refresh_level if 0 < refresh_level < n_q else n_q - 1
        self.log_n, self.n = log_n, 1 << log_n
        self.n_q, self.n_p, self.alpha = n_q, n_p, n_p
        self.dnum = (n_q + n_p - 1) // n_p
        self.log_scale, self.dg, self.df, self.min_level = log_scale, dg, df, min_level
        self.slots = self.n // 2

    @classmethod
    def from_params(cls, params):
        keys = ("log_n", "n_q", "q_bits", "n_p", "p_bits", "log_scale", "dg", "df", "min_level", "refresh_level")
        o = cls(**{k: params[k] for k in keys if k in params})
        if params.get("h", 0) or params.get("boot_K", 0):
            o.set_boot(params.get("h", 0), params.get("boot_K", 0), params.get("boot_r", 0),
                       params.get("boot_deg", 1), params.get("boot_ratio", 1), params.get("boot_groups", 1),
                       params.get("boot_refresh", 0))
            if params.get("boot_sparse", 0) and o.boot_out_level() >= 0:
                o.set_boot_sparse(params["boot_sparse"])
        return o

    # -- bootstrapping -------------------------------------------------------
    def set_boot(self, h, K, r, deg, ratio, groups, mode):
        """Sparse secret weight h and bootstrapping parameters (before keygen).
        Returns the level of a bootstrapped ciphertext (-1: chain too short)."""
        self.boot = dict(h=h, K=K, r=r, deg=deg, ratio=ratio, groups=groups, mode=mode)
        out = self.lib.orc_set_boot(self.h, int(h), int(K), int(r), int(deg), int(ratio), int(groups), int(mode))
        if mode and out >= 0:
            self.refresh_level = out
        return out

    def set_boot_sparse(self, n):
        """Slots [0, n) kept by the sparse-slot bootstrap (0: off); after set_boot."""
        if self.lib.orc_set_boot_sparse(self.h, int(n)) != 0:
            raise ValueError(f"sparse-slot bootstrap cannot take n = {n}")
        self.boot_sparse = int(n)

    def boot_out_level(self):
        return self.lib.orc_boot_out_level(self.h)

    def boot_steps(self):
        out = np.zeros(4096, dtype=np.int64)
        k = self.lib.orc_boot_steps(self.h, _p(out, C.c_int64), len(out))
        return [int(v) for v in out[:k]]

    def boot_cheb(self):
        out = np.zeros(self.boot["deg"] + 1)
        self.lib.orc_boot_cheb(self.h, _p(out, C.c_double))
        return out

    def boot_group_apply(self, inverse, g, v):
        v = np.asarray(v, dtype=np.complex128)
        vr = np.ascontiguousarray(v.real)
        vi = np.ascontiguousarray(v.imag)
        ore = np.zeros(self.slots)
        oim = np.zeros(self.slots)
        self.lib.orc_boot_group_apply(self.h, int(inverse), int(g), _p(vr, C.c_double), _p(vi, C.c_double),
                                      _p(ore, C.c_double), _p(oim, C.c_double))
        return ore + 1j * oim

    def boot_sparse_apply(self, inverse, v):
        """The sparse-slot CoeffToSlot (1) or SlotToCoeff (0) as a slot map on one
        2n period (v: 2n complex values)."""
        v = np.asarray(v, dtype=np.complex128)
        vr = np.ascontiguousarray(v.real)
        vi = np.ascontiguousarray(v.imag)
        ore = np.zeros(len(v))
        oim = np.zeros(len(v))
        self.lib.orc_boot_sparse_apply(self.h, int(inverse), _p(vr, C.c_double), _p(vi, C.c_double),
                                       _p(ore, C.c_double), _p(oim, C.c_double))
        return ore + 1j * oim

    def boot_transform_sparse(self, ct, inverse):
        """The sparse-slot CoeffToSlot (1) or SlotToCoeff (0), groups - 1 levels."""
        return self._wrap(self.lib.orc_boot_transform_sparse(self.h, ct.h, int(inverse)))

    def bootstrap_sparse(self, ct):
        """Bootstrap keeping slots [0, n) (n = boot_sparse), repeated with period n."""
        return self._wrap(self.lib.orc_bootstrap_sparse(self.h, ct.h))

    def bootstrap_packed(self, cts):
        """Refresh several ciphertexts read only on slots [0, W) (W = boot_sparse)
        through shared full-slot bootstraps: output j holds input j's slots
        [0, W) there and the other inputs' windows elsewhere."""
        k = len(cts)
        arr = (C.c_void_p * k)(*[c.h for c in cts])
        out = (C.c_void_p * k)()
        self.lib.orc_bootstrap_packed(self.h, arr, k, out)
        return [self._wrap(out[i]) for i in range(k)]

    def mod_raise(self, ct):
        return self._wrap(self.lib.orc_mod_raise(self.h, ct.h))

    def mul_monomial_half(self, ct, neg):
        return self._wrap(self.lib.orc_mul_monomial_half(self.h, ct.h, int(neg)))

    def eval_mod(self, ct):
        return self._wrap(self.lib.orc_eval_mod(self.h, ct.h))

    def boot_transform(self, ct, inverse):
        """CoeffToSlot (inverse = 1) or SlotToCoeff (inverse = 0): every group, one level each."""
        return self._wrap(self.lib.orc_boot_transform(self.h, ct.h, int(inverse)))

    def bootstrap(self, ct):
        return self._wrap(self.lib.orc_bootstrap(self.h, ct.h))

    def encode_complex(self, z, scale):
        z = np.asarray(z, dtype=np.complex128)
        zr = np.ascontiguousarray(z.real)
        zi = np.ascontiguousarray(z.imag)
        out = np.zeros(self.n, dtype=np.int64)
        self.lib.orc_encode_complex(self.h, _p(zr, C.c_double), _p(zi, C.c_double), len(z), float(scale),
                                    _p(out, C.c_int64))
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_destroy(self.h)
            self.h = None

    # -- context -------------------------------------------------------------
    @property
    def primes(self):
        out = np.zeros(self.n_q + self.n_p, dtype=np.uint64)
        self.lib.orc_primes(self.h, _p(out, C.c_uint64))
        return out

    def psi(self, t):
        return int(self.lib.orc_psi(self.h, t))

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        self.lib.orc_counters(self.h, _p(out, C.c_int64))
        names = ["sign", "rotate", "relin", "key_switch", "refresh", "poly", "max"]
        return {k: int(out[i]) for i, k in enumerate(names)}

    def reset_counters(self):
        self.lib.orc_reset_counters(self.h)

    def set_textbook(self, on):
        """Evaluate products the textbook way (Sec. 2.2: tensor, relinearise,
        rescale, six key switches per Sign polynomial) instead of the merged
        relinearise-and-rescale with lazy relinearisation (five)."""
        self.lib.orc_set_textbook(self.h, int(bool(on)))

    def galois_elt(self, step):
        return int(self.lib.orc_galois_elt(self.h, int(step)))

    # -- polynomial primitives ----------------------------------------------
    def ring_mul(self, t, a, b):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.zeros(self.n, dtype=np.uint64)
        self.lib.orc_ring_mul(self.h, t, _p(a, C.c_uint64), _p(b, C.c_uint64), _p(out, C.c_uint64))
        return out

    def ntt_roundtrip(self, t, a):
        a = np.array(a, dtype=np.uint64, copy=True)
        self.lib.orc_ntt_roundtrip(self.h, t, _p(a, C.c_uint64))
        return a

    def automorph(self, t, a, g):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        out = np.zeros(self.n, dtype=np.uint64)
        self.lib.orc_automorph(self.h, t, _p(a, C.c_uint64), int(g), _p(out, C.c_uint64))
        return out

    # -- encoding ------------------------------------------------------------
    def encode(self, z, scale):
        z = np.ascontiguousarray(z, dtype=np.float64)
        out = np.zeros(self.n, dtype=np.int64)
        self.lib.orc_encode(self.h, _p(z, C.c_double), len(z), float(scale), _p(out, C.c_int64))
        return out

    def decode(self, m, scale, nslots):
        m = np.ascontiguousarray(m, dtype=np.int64)
        out = np.zeros(nslots)
        self.lib.orc_decode(self.h, _p(m, C.c_int64), float(scale), nslots, _p(out, C.c_double))
        return out

    def layout(self, logits):
        logits = np.ascontiguousarray(logits, dtype=np.float64)
        K, Cc = logits.shape
        out = np.zeros(self.slots)
        self.lib.orc_layout(self.h, _p(logits, C.c_double), K, Cc, _p(out, C.c_double))
        return out

    # -- keys ----------------------------------------------------------------
    def keygen(self, seed, steps=()):
        st = np.ascontiguousarray(list(steps) or [0], dtype=np.int64)
        self.lib.orc_keygen(self.h, int(seed), _p(st, C.c_int64), len(steps))

    def gen_secret(self, seed):
        self.lib.orc_gen_secret(self.h, int(seed))

    def secret(self):
        out = np.zeros(self.n, dtype=np.int64)
        self.lib.orc_get_secret(self.h, _p(out, C.c_int64))
        return out

    def key_limb(self, g, digit, which, t):
        out = np.zeros(self.n, dtype=np.uint64)
        rc = self.lib.orc_get_key(self.h, int(g), digit, which, t, _p(out, C.c_uint64))
        if rc != 0:
            raise KeyError((g, digit, which, t))
        return out

    # -- ciphertexts -----------------------------------------------------------
    def _wrap(self, h):
        return Ct(self, h)

    def ct_import(self, data, scale):
        data = np.ascontiguousarray(data, dtype=np.uint64)
        level = data.shape[1] - 1
        return self._wrap(self.lib.orc_ct_import(self.h, _p(data, C.c_uint64), level, float(scale)))

    def encrypt(self, m, scale, seed):
        m = np.ascontiguousarray(m, dtype=np.int64)
        return self._wrap(self.lib.orc_encrypt(self.h, _p(m, C.c_int64), float(scale), int(seed)))

    def encrypt_logits(self, logits, seed):
        logits = np.ascontiguousarray(logits, dtype=np.float64)
        K, Cc = logits.shape
        return self._wrap(self.lib.orc_encrypt_logits(self.h, _p(logits, C.c_double), K, Cc, int(seed)))

    def decrypt(self, ct):
        out = np.zeros(self.n, dtype=np.int64)
        self.lib.orc_decrypt(self.h, ct.h, _p(out, C.c_int64))
        return out

    def decrypt_decode(self, ct, nslots):
        out = np.zeros(nslots)
        self.lib.orc_decrypt_decode(self.h, ct.h, nslots, _p(out, C.c_double))
        return out

    # -- homomorphic operations ---------------------------------------------
    def add(self, a, b):
        return self._wrap(self.lib.orc_add(self.h, a.h, b.h))

    def sub(self, a, b):
        return self._wrap(self.lib.orc_sub(self.h, a.h, b.h))

    def add_const(self, a, v):
        return self._wrap(self.lib.orc_add_const(self.h, a.h, float(v)))

    def rescale(self, a):
        return self._wrap(self.lib.orc_rescale(self.h, a.h))

    def lower(self, a, level):
        return self._wrap(self.lib.orc_lower(self.h, a.h, int(level)))

    def mul_const(self, a, v, target):
        return self._wrap(self.lib.orc_mul_const(self.h, a.h, float(v), float(target)))

    def mul_plain(self, a, v, target):
        v = np.ascontiguousarray(v, dtype=np.float64)
        return self._wrap(self.lib.orc_mul_plain(self.h, a.h, _p(v, C.c_double), len(v), float(target)))

    def mul_relin(self, a, b):
        return self._wrap(self.lib.orc_mul_relin(self.h, a.h, b.h))

    def mul_relin_rescale(self, a, b):
        return self._wrap(self.lib.orc_mul_relin_rescale(self.h, a.h, b.h))

    def rotate(self, a, step):
        return self._wrap(self.lib.orc_rotate(self.h, a.h, int(step)))

    def rotate_hoisted(self, a, steps):
        """RotL(a, s) for every s in steps, sharing one ModUp of a's c1."""
        st = np.ascontiguousarray(steps, dtype=np.int64)
        out = (C.c_void_p * len(st))()
        self.lib.orc_rotate_hoisted(self.h, a.h, _p(st, C.c_int64), len(st), out)
        return [self._wrap(v) for v in out]

    def refresh(self, a, seed, index):
        return self._wrap(self.lib.orc_refresh(self.h, a.h, int(seed), int(index)))

    def key_switch(self, g, d):
        d = np.ascontiguousarray(d, dtype=np.uint64)
        level = d.shape[0] - 1
        u0 = np.zeros_like(d)
        u1 = np.zeros_like(d)
        self.lib.orc_key_switch(self.h, int(g), _p(d, C.c_uint64), level, _p(u0, C.c_uint64), _p(u1, C.c_uint64))
        return u0, u1

    def key_switch_raw(self, g, d):
        """ModUp + inner product only: (acc0, acc1) over Q_level then the special primes."""
        d = np.ascontiguousarray(d, dtype=np.uint64)
        level = d.shape[0] - 1
        shape = (level + 1 + self.n_p, self.n)
        a0 = np.zeros(shape, np.uint64)
        a1 = np.zeros(shape, np.uint64)
        self.lib.orc_key_switch_raw(self.h, int(g), _p(d, C.c_uint64), level, _p(a0, C.c_uint64), _p(a1, C.c_uint64))
        return a0, a1

    def relin_rescale3(self, d, scale):
        """Relinearise-and-rescale of a degree-2 ciphertext d[3, level+1, N]."""
        d = np.ascontiguousarray(d, dtype=np.uint64)
        return self._wrap(self.lib.orc_relin_rescale3(self.h, _p(d, C.c_uint64), d.shape[1] - 1, float(scale)))

    def lincomb(self, a, va, b, vb, target, rescale=True):
        return self._wrap(self.lib.orc_lincomb(self.h, a.h, float(va), b.h if b is not None else None, float(vb),
                                               float(target), int(bool(rescale))))

    def eval_odd9(self, x, coef, gain, target):
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        return self._wrap(self.lib.orc_eval_odd9(self.h, x.h, _p(coef, C.c_double), float(gain), float(target)))

    def eval_argmax_phoenix(self, ct, K, Cc, d_min, d_max, refresh_seed):
        """The comparison path (Phoenix): C Signs and C rotations."""
        return self._wrap(self.lib.orc_eval_argmax_phoenix(self.h, ct.h, int(K), int(Cc), float(d_min), float(d_max),
                                                           int(refresh_seed)))

    def packed_shape(self, shapes):
        """(blocks per ciphertext, K', C', block size) for a group of (K, C) shapes."""
        Ks = np.ascontiguousarray([k for k, _ in shapes], dtype=np.int32)
        Cs = np.ascontiguousarray([c for _, c in shapes], dtype=np.int32)
        out = np.zeros(3, dtype=np.int32)
        nb = self.lib.orc_packed_shape(self.h, len(shapes), _p(Ks, C.c_int), _p(Cs, C.c_int), _p(out, C.c_int))
        return int(nb), int(out[0]), int(out[1]), int(out[2])

    def encrypt_packed(self, blocks, seed):
        """blocks: list of K_b x C_b logit arrays, packed one per slot block."""
        Ks, Cs, flat = _packed_args(blocks)
        return self._wrap(self.lib.orc_encrypt_packed(self.h, len(blocks), _p(flat, C.c_double), _p(Ks, C.c_int),
                                                      _p(Cs, C.c_int), int(seed)))

    def eval_argmax_packed(self, ct, shapes, d_min, d_max, refresh_seed):
        Ks = np.ascontiguousarray([k for k, _ in shapes], dtype=np.int32)
        Cs = np.ascontiguousarray([c for _, c in shapes], dtype=np.int32)
        lo = np.ascontiguousarray(d_min, dtype=np.float64)
        hi = np.ascontiguousarray(d_max, dtype=np.float64)
        return self._wrap(self.lib.orc_eval_argmax_packed(self.h, ct.h, len(shapes), _p(Ks, C.c_int), _p(Cs, C.c_int),
                                                          _p(lo, C.c_double), _p(hi, C.c_double), int(refresh_seed)))

    def decrypt_packed(self, ct, shapes):
        """Each block's decrypted z[:C_b]."""
        nb, kp, cp, bsz = self.packed_shape(shapes)
        z = self.decrypt_decode(ct, len(shapes) * bsz)
        return [z[b * bsz:b * bsz + c] for b, (_, c) in enumerate(shapes)]

    def eval_argmax(self, ct, K, Cc, d_min, d_max, refresh_seed):
        return self._wrap(self.lib.orc_eval_argmax(self.h, ct.h, int(K), int(Cc), float(d_min), float(d_max),
                                                   int(refresh_seed)))


def _packed_args(blocks):
    Ks = np.ascontiguousarray([np.asarray(l).shape[0] for l in blocks], dtype=np.int32)
    Cs = np.ascontiguousarray([np.asarray(l).shape[1] for l in blocks], dtype=np.int32)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(l, dtype=np.float64).ravel() for l in blocks]))
    return Ks, Cs, flat


def argmax_rotation_steps(k_max, c_max, slots):
    """RotL amounts Algorithm 1 uses for any K <= k_max, C <= c_max: the prompt
    sum C'*2^i, the duplication RotR(C') = RotL(slots - C'), QuickMax 2^i."""
    steps = set()
    cp_max = 1 << max(0, (c_max - 1).bit_length())
    kp_max = 1 << max(0, (k_max - 1).bit_length())
    cp = 1
    while cp <= cp_max:
        steps.add(slots - cp)
        i = 1
        while cp * i < cp * kp_max:
            steps.add(cp * i)
            i <<= 1
        cp <<= 1
    j = 1
    while j < cp_max:
        steps.add(j)
        j <<= 1
    steps.discard(slots)
    return sorted(steps)
