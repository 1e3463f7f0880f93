"""Python binding of libsecpe.so (include/secpe.h): argument marshalling only.

Every step runs in the library's HIP kernels; PyTorch provides device memory
(float64 CUDA tensors holding exact residues) and the stream.  There is no CPU
fallback: a missing library or GPU raises.
"""
import ctypes as C
import os

import numpy as np

from .build import lib_path

_lib = None

SECPE_GRAPH = 1


class SecpeError(RuntimeError):
    pass


class _Params(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("log_n", "n_q", "q_bits", "n_p", "p_bits", "log_scale", "dg", "df", "min_level",
                                       "refresh_level")]


class _BootParams(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("secret_h", "K", "r", "deg", "ratio", "groups", "refresh", "sparse_slots",
                                       "pack_min")]


# the step value keygen takes for the conjugation key
STEP_CONJUGATE = -(1 << 63)


class _Ct(C.Structure):
    _fields_ = [("data", C.c_void_p), ("level", C.c_int), ("scale", C.c_double)]


def load():
    """Load the built library (build it first with build.build())."""
    global _lib
    if _lib is not None:
        return _lib
    # torch's bundled HIP runtime (soname libamdhip64.so.7) must be the one the
    # library binds to, so load torch before the library
    import torch  # noqa: F401
    path = lib_path()
    if not os.path.exists(path):
        raise SecpeError(f"{path} is missing: run paper_2502_00847_amd.build.build() first")
    lib = C.CDLL(path)
    vp, i32, i64, u64, dbl, sz = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double, C.c_size_t
    P = C.POINTER
    ct = P(_Ct)
    sig = {
        "secpe_last_error": (C.c_char_p, []),
        "secpe_strerror": (C.c_char_p, [i32]),
        "secpe_ctx_create": (i32, [P(_Params), i32, vp, P(vp)]),
        "secpe_ctx_destroy": (None, [vp]),
        "secpe_primes": (i32, [vp, P(u64), i32]),
        "secpe_slots": (i32, [vp]),
        "secpe_ct_bytes": (sz, [vp]),
        "secpe_sk_bytes": (sz, [vp]),
        "secpe_key_bytes": (sz, [vp]),
        "secpe_galois_elt": (u64, [vp, i64]),
        "secpe_argmax_steps": (i32, [vp, i32, i32, P(i64), i32]),
        "secpe_keygen": (i32, [vp, u64, P(i64), i32, vp, vp]),
        "secpe_key_owner_create": (i32, [vp, vp, P(vp)]),
        "secpe_key_owner_destroy": (None, [vp]),
        "secpe_encrypt": (i32, [vp, vp, P(dbl), i32, i32, u64, ct]),
        "secpe_encrypt_coeffs": (i32, [vp, vp, P(i64), dbl, u64, ct]),
        "secpe_decrypt": (i32, [vp, vp, ct, i32, P(dbl), P(i32)]),
        "secpe_decrypt_coeffs": (i32, [vp, vp, ct, P(i64)]),
        "secpe_workspace_bytes": (sz, [vp, i32, P(i32), P(i32)]),
        "secpe_eval_argmax": (i32, [vp, vp, ct, i32, i32, dbl, dbl, u64, vp, sz, ct]),
        "secpe_eval_argmax_noalloc": (i32, [vp, vp, ct, i32, i32, dbl, dbl, u64, ct]),
        "secpe_eval_argmax_batch": (i32, [vp, vp, i32, ct, P(i32), P(i32), P(dbl), P(dbl), P(u64), vp, sz, ct, i32]),
        "secpe_counters": (i32, [vp, P(i64)]),
        "secpe_ct_export": (i32, [vp, ct, P(u64)]),
        "secpe_ct_import": (i32, [vp, P(u64), i32, dbl, ct]),
        "secpe_key_export": (i32, [vp, vp, i32, i32, i32, i32, P(u64)]),
        "secpe_sk_export": (i32, [vp, vp, P(i64)]),
        "secpe_sync": (i32, [vp]),
        "secpe_op_workspace_bytes": (sz, [vp]),
        "secpe_op_add": (i32, [vp, ct, ct, ct]),
        "secpe_op_sub": (i32, [vp, ct, ct, ct]),
        "secpe_op_add_const": (i32, [vp, ct, dbl, ct]),
        "secpe_op_mul_const": (i32, [vp, ct, dbl, dbl, vp, sz, ct]),
        "secpe_op_lincomb": (i32, [vp, ct, dbl, ct, dbl, dbl, i32, vp, sz, ct]),
        "secpe_packed_shape": (i32, [vp, i32, P(i32), P(i32), P(i32)]),
        "secpe_phoenix_steps": (i32, [vp, i32, i32, P(i64), i32]),
        "secpe_phoenix_workspace_bytes": (sz, [vp, i32, i32]),
        "secpe_eval_argmax_phoenix": (i32, [vp, vp, ct, i32, i32, dbl, dbl, u64, vp, sz, ct]),
        "secpe_encrypt_packed": (i32, [vp, vp, i32, P(dbl), P(i32), P(i32), u64, ct]),
        "secpe_packed_workspace_bytes": (sz, [vp, i32, P(i32), P(i32), P(i32)]),
        "secpe_eval_argmax_packed": (i32, [vp, vp, i32, ct, P(i32), P(i32), P(i32), P(dbl), P(dbl), P(u64), vp, sz,
                                           ct]),
        "secpe_autotune": (i32, [vp, vp, i32, ct, P(i32), P(i32), P(dbl), P(dbl), P(u64), vp, sz, ct, P(i32),
                                 P(dbl), i32]),
        "secpe_op_mul_plain": (i32, [vp, ct, P(dbl), i32, dbl, vp, sz, ct]),
        "secpe_op_rescale": (i32, [vp, ct, vp, sz, ct]),
        "secpe_op_mul_relin": (i32, [vp, ct, ct, vp, sz, ct]),
        "secpe_op_mul_relin_rescale": (i32, [vp, ct, ct, vp, sz, ct]),
        "secpe_op_rotate": (i32, [vp, ct, i64, vp, sz, ct]),
        "secpe_op_refresh": (i32, [vp, vp, ct, u64, u64, vp, sz, ct]),
        "secpe_op_eval_odd9": (i32, [vp, ct, P(dbl), dbl, dbl, vp, sz, ct]),
        "secpe_op_key_switch": (i32, [vp, i32, P(u64), i32, vp, sz, P(u64), P(u64)]),
        "secpe_op_ntt": (i32, [vp, i32, P(u64), i32, P(u64), P(u64)]),
        "secpe_op_ring_mul": (i32, [vp, i32, P(u64), P(u64), P(u64)]),
        "secpe_op_encode": (i32, [vp, P(dbl), i32, dbl, P(i64)]),
        "secpe_profile_begin": (i32, [vp, i32]),
        "secpe_profile_end": (i32, [vp, P(i64), P(dbl), P(i64), P(i64)]),
        "secpe_keyswitch_traffic": (i32, [vp, P(i64)]),
        "secpe_set_schedule": (i32, [vp, i32]),
        "secpe_profile_segments": (i32, [vp, P(dbl), i32]),
        "secpe_ntt_cts": (i32, [vp, ct, i32, i32]),
        "secpe_rotate_workspace_bytes": (sz, [vp, i32]),
        "secpe_rotate_batch": (i32, [vp, i32, ct, P(i64), vp, sz, ct]),
        "secpe_server_create": (i32, [vp, vp, vp, sz, i32, P(vp)]),
        "secpe_server_destroy": (None, [vp]),
        "secpe_server_request_bytes": (sz, [vp, i32, i32]),
        "secpe_server_submit": (i32, [vp, ct, i32, i32, dbl, dbl, u64, vp, P(u64)]),
        "secpe_server_step": (i32, [vp, i32, P(i32), P(u64), P(i32), P(dbl), P(i32), P(i32)]),
        "secpe_server_launch": (i32, [vp]),
        "secpe_keys_share": (i32, [vp, vp]),
        "secpe_server_ready": (i32, [vp]),
        "secpe_server_collect": (i32, [vp, i32, P(i32), P(u64), P(i32), P(dbl), P(i32), P(i32)]),
        "secpe_set_boot": (i32, [vp, P(_BootParams), P(i32)]),
        "secpe_boot_steps": (i32, [vp, P(i64), i32]),
        "secpe_boot_key_bytes": (sz, [vp]),
        "secpe_boot_setup": (i32, [vp, vp, sz]),
        "secpe_bootstrap_workspace_bytes": (sz, [vp, i32]),
        "secpe_bootstrap": (i32, [vp, i32, ct, vp, sz, ct]),
        "secpe_bootstrap_sparse": (i32, [vp, i32, ct, vp, sz, ct]),
        "secpe_bootstrap_packed": (i32, [vp, i32, ct, vp, sz, ct]),
        "secpe_op_boot_step": (i32, [vp, i32, ct, vp, sz, ct]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names the library must export (those declared in include/secpe.h)."""
    return sorted(
        ["secpe_last_error", "secpe_strerror", "secpe_ctx_create", "secpe_ctx_destroy", "secpe_primes", "secpe_slots",
         "secpe_ct_bytes", "secpe_sk_bytes", "secpe_key_bytes", "secpe_galois_elt", "secpe_argmax_steps",
         "secpe_keygen", "secpe_key_owner_create", "secpe_key_owner_destroy", "secpe_encrypt", "secpe_encrypt_coeffs", "secpe_decrypt",
         "secpe_decrypt_coeffs", "secpe_workspace_bytes", "secpe_eval_argmax", "secpe_eval_argmax_noalloc", "secpe_eval_argmax_batch",
         "secpe_counters", "secpe_ct_export", "secpe_ct_import", "secpe_key_export", "secpe_sk_export",
         "secpe_sync", "secpe_op_workspace_bytes", "secpe_op_add", "secpe_op_sub", "secpe_op_add_const",
         "secpe_op_mul_const", "secpe_op_lincomb", "secpe_autotune", "secpe_set_schedule", "secpe_packed_shape", "secpe_encrypt_packed",
         "secpe_packed_workspace_bytes", "secpe_eval_argmax_packed", "secpe_phoenix_steps",
         "secpe_phoenix_workspace_bytes", "secpe_eval_argmax_phoenix", "secpe_op_mul_plain", "secpe_op_rescale", "secpe_op_mul_relin",
         "secpe_op_mul_relin_rescale", "secpe_op_rotate", "secpe_op_refresh", "secpe_op_eval_odd9",
         "secpe_op_key_switch", "secpe_op_ntt", "secpe_op_ring_mul", "secpe_op_encode", "secpe_profile_begin",
         "secpe_profile_end", "secpe_profile_segments", "secpe_keyswitch_traffic", "secpe_ntt_cts", "secpe_rotate_workspace_bytes", "secpe_rotate_batch",
         "secpe_server_create", "secpe_server_destroy", "secpe_server_request_bytes", "secpe_server_submit",
         "secpe_server_step", "secpe_server_launch", "secpe_server_ready", "secpe_keys_share",
         "secpe_server_collect", "secpe_set_boot", "secpe_boot_steps", "secpe_boot_key_bytes", "secpe_boot_setup",
         "secpe_bootstrap_workspace_bytes", "secpe_bootstrap", "secpe_bootstrap_sparse", "secpe_bootstrap_packed", "secpe_op_boot_step"])


def _p(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


class Ciphertext:
    """Device ciphertext: a float64 CUDA tensor [2, n_q, N] (NTT domain), level, scale."""

    def __init__(self, buf, level, scale):
        self.buf = buf
        self.level = int(level)
        self.scale = float(scale)

    def _c(self):
        return _Ct(C.c_void_p(self.buf.data_ptr()), self.level, self.scale)


class KeyOwner:
    """The key owner's handle (secpe_key_owner): names the secret for the
    refresh stand-in of bootstrapping.  Evaluations that may refresh take it
    explicitly; without one they stop with SECPE_ENOLEVEL."""

    def __init__(self, ctx, sk):
        self.lib = ctx.lib
        self.sk = sk
        h = C.c_void_p()
        ctx._check(self.lib.secpe_key_owner_create(ctx.h, C.c_void_p(sk.data_ptr()), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.secpe_key_owner_destroy(self.h)
            self.h = None


def _owner(owner):
    return owner.h if owner is not None else None


class Context:
    """RNS-CKKS context on one GPU (params: a dict with the secpe_params fields)."""

    def __init__(self, params, device=0):
        import torch
        if not torch.cuda.is_available():
            raise SecpeError("no GPU visible: the HIP library needs an MI355X")
        self.torch = torch
        self.lib = load()
        self.device = device
        torch.cuda.set_device(device)
        self.stream = torch.cuda.Stream(device=device)
        p = _Params(**{k: int(params.get(k, 0)) for k, _ in _Params._fields_})
        h = C.c_void_p()
        self._check(self.lib.secpe_ctx_create(C.byref(p), device, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.params = dict(params)
        self.N = 1 << params["log_n"]
        self.n_q, self.n_p = params["n_q"], params["n_p"]
        self.slots = self.N // 2
        self.sk = None
        self.evk = None
        self.boot_out_level = -1
        if params.get("h", 0) or params.get("boot_K", 0):
            self.set_boot(params.get("h", 0), params.get("boot_K", 0), params.get("boot_r", 0),
                          params.get("boot_deg", 1), params.get("boot_ratio", 1), params.get("boot_groups", 1),
                          params.get("boot_refresh", 0), params.get("boot_sparse", 0), params.get("boot_pack_min", 0))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.secpe_ctx_destroy(self.h)
            self.h = None

    def _check(self, rc):
        if rc != 0:
            raise SecpeError(f"secpe error {rc}: {self.lib.secpe_last_error().decode()}")

    def _empty(self, nbytes):
        with self.torch.cuda.stream(self.stream):
            return self.torch.empty(max(1, (nbytes + 7) // 8), dtype=self.torch.float64, device=f"cuda:{self.device}")

    # -- sizes and tables ------------------------------------------------------
    @property
    def primes(self):
        out = np.zeros(self.n_q + self.n_p, dtype=np.uint64)
        self.lib.secpe_primes(self.h, _p(out, C.c_uint64), len(out))
        return out

    def ct_bytes(self):
        return self.lib.secpe_ct_bytes(self.h)

    def new_ct(self):
        return Ciphertext(self._empty(self.ct_bytes()), -1, 0.0)

    def galois_elt(self, step):
        return int(self.lib.secpe_galois_elt(self.h, int(step)))

    def argmax_steps(self, k_max, c_max):
        out = np.zeros(256, dtype=np.int64)
        n = self.lib.secpe_argmax_steps(self.h, k_max, c_max, _p(out, C.c_int64), len(out))
        return [int(v) for v in out[:n]]

    # -- keys ------------------------------------------------------------------
    def keygen(self, seed, steps):
        """Client key generation: the secret (kept here for the client's
        encrypt and decrypt calls) and the switching keys the context evaluates
        with.  The context itself never holds the secret."""
        steps = list(steps)
        self.sk = self._empty(self.lib.secpe_sk_bytes(self.h))
        self.evk = self._empty(self.lib.secpe_key_bytes(self.h) * (1 + len(steps)))
        st = np.ascontiguousarray(steps or [0], dtype=np.int64)
        self._check(self.lib.secpe_keygen(self.h, int(seed), _p(st, C.c_int64), len(steps),
                                          C.c_void_p(self.sk.data_ptr()), C.c_void_p(self.evk.data_ptr())))
        self.steps = steps
        return self.sk, self.evk

    def key_owner(self, sk=None):
        """A key-owner handle for the client's secret (or the given one)."""
        return KeyOwner(self, self.sk if sk is None else sk)

    def share_keys(self, other):
        """Evaluate with other's switching keys (same parameters and device);
        this context keeps its own stream.  The client-side secret reference is
        copied for this binding's encrypt and decrypt conveniences only."""
        self._check(self.lib.secpe_keys_share(self.h, other.h))
        self.sk, self.evk, self.steps = other.sk, other.evk, other.steps

    # -- bootstrapping -----------------------------------------------------------
    def set_boot(self, h, K, r, deg, ratio, groups, refresh, sparse_slots=0, pack_min=0):
        """Sparse secret weight and bootstrapping parameters (before keygen);
        sparse_slots = n > 0 adds the sparse-slot bootstrap of slots [0, n);
        pack_min = k >= 2 packs refreshes of at least k such ciphertexts into
        shared full-slot bootstraps."""
        bp = _BootParams(int(h), int(K), int(r), int(deg), int(ratio), int(groups), int(refresh), int(sparse_slots),
                         int(pack_min))
        lvl = C.c_int(-1)
        self._check(self.lib.secpe_set_boot(self.h, C.byref(bp), C.byref(lvl)))
        self.boot_out_level = lvl.value
        return lvl.value

    def boot_steps(self):
        out = np.zeros(4096, dtype=np.int64)
        n = self.lib.secpe_boot_steps(self.h, _p(out, C.c_int64), len(out))
        if n < 0:
            self._check(n)
        return [int(v) for v in out[:n]]

    def boot_setup(self):
        """Encode the linear-transform plaintexts (after keygen)."""
        nb = self.lib.secpe_boot_key_bytes(self.h)
        self.boot_keys = self._empty(nb)
        self._check(self.lib.secpe_boot_setup(self.h, C.c_void_p(self.boot_keys.data_ptr()), nb))

    def bootstrap_workspace(self, n):
        nb = self.lib.secpe_bootstrap_workspace_bytes(self.h, int(n))
        if nb == 0:
            raise SecpeError(self.lib.secpe_last_error().decode())
        return self._empty(nb)

    def bootstrap(self, cts, ws=None, outs=None, sparse=False, packed=False):
        """Bootstrap every ciphertext; sparse: keep slots [0, sparse_slots) only;
        packed: the window-packed bootstrap (secpe_bootstrap_packed)."""
        n = len(cts)
        ws = self.bootstrap_workspace(n) if ws is None else ws
        outs = [self.new_ct() for _ in range(n)] if outs is None else outs
        ins = (_Ct * n)(*[c._c() for c in cts])
        os_ = (_Ct * n)(*[o._c() for o in outs])
        fn = (self.lib.secpe_bootstrap_packed if packed else
              self.lib.secpe_bootstrap_sparse if sparse else self.lib.secpe_bootstrap)
        self._check(fn(self.h, n, ins, C.c_void_p(ws.data_ptr()), ws.numel() * 8, os_))
        for o, c in zip(outs, os_):
            o.level, o.scale = c.level, c.scale
        return outs

    def boot_step(self, step, a):
        """0 ModRaise, 1 CoeffToSlot, 2 SlotToCoeff, 3 EvalMod, 4 times i, 5 times -i,
        6 and 7 the sparse-slot CoeffToSlot and SlotToCoeff."""
        if getattr(self, "_bws", None) is None:
            self._bws = self.bootstrap_workspace(1)
        out = self.new_ct()
        c = out._c()
        self._check(self.lib.secpe_op_boot_step(self.h, int(step), C.byref(a._c()), C.c_void_p(self._bws.data_ptr()),
                                                self._bws.numel() * 8, C.byref(c)))
        out.level, out.scale = c.level, c.scale
        return out

    # -- client ------------------------------------------------------------------
    def encrypt(self, logits, seed, sk=None):
        sk = self.sk if sk is None else sk
        logits = np.ascontiguousarray(logits, dtype=np.float64)
        K, Cc = logits.shape
        ct = self.new_ct()
        c = ct._c()
        self._check(self.lib.secpe_encrypt(self.h, C.c_void_p(sk.data_ptr()), _p(logits, C.c_double), K, Cc,
                                           int(seed), C.byref(c)))
        ct.level, ct.scale = c.level, c.scale
        return ct

    def encrypt_coeffs(self, m, scale, seed, sk=None):
        sk = self.sk if sk is None else sk
        m = np.ascontiguousarray(m, dtype=np.int64)
        ct = self.new_ct()
        c = ct._c()
        self._check(self.lib.secpe_encrypt_coeffs(self.h, C.c_void_p(sk.data_ptr()), _p(m, C.c_int64), float(scale),
                                                  int(seed), C.byref(c)))
        ct.level, ct.scale = c.level, c.scale
        return ct

    def decrypt(self, ct, nslots, sk=None):
        sk = self.sk if sk is None else sk
        z = np.zeros(nslots)
        idx = C.c_int(0)
        c = ct._c()
        self._check(self.lib.secpe_decrypt(self.h, C.c_void_p(sk.data_ptr()), C.byref(c), nslots,
                                           _p(z, C.c_double), C.byref(idx)))
        return z, int(idx.value)

    # -- the comparison path (Phoenix) -------------------------------------------
    def phoenix_steps(self, k_max, c):
        out = np.zeros(1024, dtype=np.int64)
        n = self.lib.secpe_phoenix_steps(self.h, int(k_max), int(c), _p(out, C.c_int64), len(out))
        if n < 0:
            self._check(n)
        return [int(v) for v in out[:n]]

    def eval_argmax_phoenix(self, ct, K, Cc, d_min, d_max, refresh_seed, ws=None, out=None, owner=None):
        if ws is None:
            nb = self.lib.secpe_phoenix_workspace_bytes(self.h, int(K), int(Cc))
            if nb == 0:
                raise SecpeError(self.lib.secpe_last_error().decode())
            ws = self._empty(nb)
        out = self.new_ct() if out is None else out
        c = out._c()
        self._check(self.lib.secpe_eval_argmax_phoenix(self.h, _owner(owner), C.byref(ct._c()), int(K), int(Cc),
                                                       float(d_min), float(d_max), int(refresh_seed),
                                                       C.c_void_p(ws.data_ptr()), ws.numel() * 8, C.byref(c)))
        out.level, out.scale = c.level, c.scale
        return out

    # -- slot-packed Argmax ------------------------------------------------------
    def packed_shape(self, shapes):
        """(blocks per ciphertext, K', C', block size) for a group of (K, C) shapes."""
        Ks = np.ascontiguousarray([k for k, _ in shapes], dtype=np.int32)
        Cs = np.ascontiguousarray([c for _, c in shapes], dtype=np.int32)
        out = np.zeros(3, dtype=np.int32)
        per = self.lib.secpe_packed_shape(self.h, len(shapes), _p(Ks, C.c_int), _p(Cs, C.c_int), _p(out, C.c_int))
        if per < 0:
            self._check(per)
        return int(per), int(out[0]), int(out[1]), int(out[2])

    def encrypt_packed(self, blocks, seed, sk=None):
        """blocks: list of K_b x C_b logit arrays, one query per slot block."""
        sk = self.sk if sk is None else sk
        Ks = np.ascontiguousarray([np.asarray(b).shape[0] for b in blocks], dtype=np.int32)
        Cs = np.ascontiguousarray([np.asarray(b).shape[1] for b in blocks], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(b, dtype=np.float64).ravel() for b in blocks]))
        ct = self.new_ct()
        c = ct._c()
        self._check(self.lib.secpe_encrypt_packed(self.h, C.c_void_p(sk.data_ptr()), len(blocks), _p(flat, C.c_double),
                                                  _p(Ks, C.c_int), _p(Cs, C.c_int), int(seed), C.byref(c)))
        ct.level, ct.scale = c.level, c.scale
        return ct

    def _packed_arrays(self, groups):
        nb = np.ascontiguousarray([len(g) for g in groups], dtype=np.int32)
        Ks = np.ascontiguousarray([k for g in groups for k, _ in g], dtype=np.int32)
        Cs = np.ascontiguousarray([c for g in groups for _, c in g], dtype=np.int32)
        return nb, Ks, Cs

    def packed_workspace(self, groups):
        nb, Ks, Cs = self._packed_arrays(groups)
        n = self.lib.secpe_packed_workspace_bytes(self.h, len(groups), _p(nb, C.c_int), _p(Ks, C.c_int),
                                                  _p(Cs, C.c_int))
        if n == 0:
            raise SecpeError(self.lib.secpe_last_error().decode())
        return self._empty(n)

    def eval_argmax_packed(self, cts, groups, d_min, d_max, seeds, ws=None, outs=None, owner=None):
        """groups[i]: the (K, C) shapes packed in cts[i]; d_min, d_max: per block, concatenated."""
        n = len(cts)
        nb, Ks, Cs = self._packed_arrays(groups)
        lo = np.ascontiguousarray(d_min, dtype=np.float64)
        hi = np.ascontiguousarray(d_max, dtype=np.float64)
        sd = np.ascontiguousarray([int(s) for s in seeds], dtype=np.uint64)
        if ws is None:
            ws = self.packed_workspace(groups)
        if outs is None:
            outs = [self.new_ct() for _ in range(n)]
        cin = (_Ct * n)(*[c._c() for c in cts])
        cout = (_Ct * n)(*[c._c() for c in outs])
        self._check(self.lib.secpe_eval_argmax_packed(self.h, _owner(owner), n, cin, _p(nb, C.c_int), _p(Ks, C.c_int),
                                                      _p(Cs, C.c_int), _p(lo, C.c_double), _p(hi, C.c_double),
                                                      _p(sd, C.c_uint64), C.c_void_p(ws.data_ptr()), ws.numel() * 8,
                                                      cout))
        for o, c in zip(outs, cout):
            o.level, o.scale = c.level, c.scale
        return outs

    def decrypt_packed(self, ct, shapes, sk=None):
        """Each block's decrypted z[:C_b] and its index."""
        per, kp, cp, bsz = self.packed_shape(shapes)
        z, _ = self.decrypt(ct, len(shapes) * bsz, sk)
        out = []
        for b, (_, c) in enumerate(shapes):
            zb = z[b * bsz:b * bsz + c]
            out.append((zb, int(np.argmax(zb))))
        return out

    def decrypt_coeffs(self, ct, sk=None):
        sk = self.sk if sk is None else sk
        m = np.zeros(self.N, dtype=np.int64)
        c = ct._c()
        self._check(self.lib.secpe_decrypt_coeffs(self.h, C.c_void_p(sk.data_ptr()), C.byref(c), _p(m, C.c_int64)))
        return m

    # -- evaluation ----------------------------------------------------------------
    def workspace_bytes(self, Ks, Cs):
        Ks = np.ascontiguousarray(Ks, dtype=np.int32)
        Cs = np.ascontiguousarray(Cs, dtype=np.int32)
        n = self.lib.secpe_workspace_bytes(self.h, len(Ks), _p(Ks, C.c_int), _p(Cs, C.c_int))
        if n == 0:
            raise SecpeError(self.lib.secpe_last_error().decode())
        return n

    def workspace(self, Ks, Cs):
        return self._empty(self.workspace_bytes(Ks, Cs))

    def eval_argmax_batch(self, cts, Ks, Cs, d_min, d_max, seeds, ws=None, outs=None, graph=False, owner=None):
        n = len(cts)
        Ks = np.ascontiguousarray(Ks, dtype=np.int32)
        Cs = np.ascontiguousarray(Cs, dtype=np.int32)
        dmin = np.ascontiguousarray(d_min, dtype=np.float64)
        dmax = np.ascontiguousarray(d_max, dtype=np.float64)
        sd = np.ascontiguousarray([int(s) for s in seeds], dtype=np.uint64)
        if ws is None:
            ws = self.workspace(Ks, Cs)
        if outs is None:
            outs = [self.new_ct() for _ in range(n)]
        cin = (_Ct * n)(*[c._c() for c in cts])
        cout = (_Ct * n)(*[c._c() for c in outs])
        self._check(self.lib.secpe_eval_argmax_batch(self.h, _owner(owner), n, cin, _p(Ks, C.c_int), _p(Cs, C.c_int),
                                                     _p(dmin, C.c_double), _p(dmax, C.c_double),
                                                     _p(sd, C.c_uint64), C.c_void_p(ws.data_ptr()),
                                                     ws.numel() * 8, cout, SECPE_GRAPH if graph else 0))
        for o, c in zip(outs, cout):
            o.level, o.scale = c.level, c.scale
        return outs

    AUTOTUNE_CANDIDATES = [dict(modup_outputs_per_workgroup=2 if i & 1 else 4,
                                ntt_job_group_mib=128 if i & 2 else None,
                                fwd_col_tiles_per_workgroup=2 if i & 4 else 1,
                                inv_col_tiles_per_workgroup=2 if i & 8 else 1,
                                fwd_row_tiles_per_workgroup=2 if i & 16 else 1,
                                moddown_outputs_per_workgroup=2 if i & 32 else 4) for i in range(64)]

    def autotune(self, cts, Ks, Cs, d_min, d_max, seeds, ws, outs, owner=None):
        """Time the batch under each candidate schedule; the fastest stays set."""
        n = len(cts)
        Ks = np.ascontiguousarray(Ks, dtype=np.int32)
        Cs = np.ascontiguousarray(Cs, dtype=np.int32)
        dmin = np.ascontiguousarray(d_min, dtype=np.float64)
        dmax = np.ascontiguousarray(d_max, dtype=np.float64)
        sd = np.ascontiguousarray([int(s) for s in seeds], dtype=np.uint64)
        cin = (_Ct * n)(*[c._c() for c in cts])
        cout = (_Ct * n)(*[c._c() for c in outs])
        chosen = C.c_int(-1)
        ms = np.zeros(len(self.AUTOTUNE_CANDIDATES), dtype=np.float64)
        self._check(self.lib.secpe_autotune(self.h, _owner(owner), n, cin, _p(Ks, C.c_int), _p(Cs, C.c_int), _p(dmin, C.c_double),
                                            _p(dmax, C.c_double), _p(sd, C.c_uint64), C.c_void_p(ws.data_ptr()),
                                            ws.numel() * 8, cout, C.byref(chosen), _p(ms, C.c_double), len(ms)))
        for o, c in zip(outs, cout):
            o.level, o.scale = c.level, c.scale
        timed = [dict(c, index=i, ms=round(float(t), 3)) for i, (c, t) in enumerate(zip(self.AUTOTUNE_CANDIDATES, ms))
                 if t > 0]
        return chosen.value, timed

    def set_schedule(self, candidate):
        """Apply an autotuner candidate (knob bits) without timing."""
        self._check(self.lib.secpe_set_schedule(self.h, int(candidate)))

    def eval_argmax(self, ct, K, Cc, d_min, d_max, refresh_seed, ws=None, owner=None):
        return self.eval_argmax_batch([ct], [K], [Cc], [d_min], [d_max], [refresh_seed], ws=ws, owner=owner)[0]

    def eval_argmax_noalloc(self, ct, K, Cc, d_min, d_max, refresh_seed, out=None, owner=None):
        """The Argmax with its workspace in the library's per-GPU scratch array
        (secpe_eval_argmax_noalloc): the call allocates no device memory."""
        out = self.new_ct() if out is None else out
        c = out._c()
        self._check(self.lib.secpe_eval_argmax_noalloc(self.h, _owner(owner), C.byref(ct._c()), int(K), int(Cc),
                                                       float(d_min), float(d_max), int(refresh_seed), C.byref(c)))
        out.level, out.scale = c.level, c.scale
        return out

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        self._check(self.lib.secpe_counters(self.h, _p(out, C.c_int64)))
        names = ["sign", "rotate", "relin", "key_switch", "refresh", "poly", "max", "launches"]
        return {k: int(out[i]) for i, k in enumerate(names)}

    def sync(self):
        self._check(self.lib.secpe_sync(self.h))

    # -- measurement -------------------------------------------------------------
    PROF = dict(ntt_fwd=0, ntt_inv=1, ew=2, modup=3, moddown=4, inner=5, auto=6, spread=7, ntt_fwd_col=8,
                ntt_fwd_row=9, segments=10)

    def profile_begin(self, kind):
        self._check(self.lib.secpe_profile_begin(self.h, self.PROF[kind] if isinstance(kind, str) else int(kind)))

    def profile_end(self):
        n = C.c_int64(0)
        ms = C.c_double(0.0)
        u = C.c_int64(0)
        us = C.c_int64(0)
        self._check(self.lib.secpe_profile_end(self.h, C.byref(n), C.byref(ms), C.byref(u), C.byref(us)))
        return dict(launches=int(n.value), ms=float(ms.value), units=int(u.value), units_shared=int(us.value))

    def profile_segments(self):
        """Milliseconds between consecutive events of the last 'segments' profile."""
        ms = np.zeros(4096)
        n = self.lib.secpe_profile_segments(self.h, _p(ms, C.c_double), len(ms))
        self._check(min(n, 0))
        return [float(v) for v in ms[:n]]

    def keyswitch_traffic(self):
        """Algorithmic HBM bytes of the last evaluation's key switches (keys once per launch)."""
        b = C.c_int64(0)
        self._check(self.lib.secpe_keyswitch_traffic(self.h, C.byref(b)))
        return int(b.value)

    def ntt_cts(self, cts, inverse):
        arr = (_Ct * len(cts))(*[c._c() for c in cts])
        self._check(self.lib.secpe_ntt_cts(self.h, arr, len(cts), 1 if inverse else 0))

    def rotate_batch(self, cts, steps, ws=None, outs=None):
        n = len(cts)
        if ws is None:
            ws = self._empty(self.lib.secpe_rotate_workspace_bytes(self.h, n))
        if outs is None:
            outs = [self.new_ct() for _ in range(n)]
        st = np.ascontiguousarray(steps, dtype=np.int64)
        cin = (_Ct * n)(*[c._c() for c in cts])
        cout = (_Ct * n)(*[c._c() for c in outs])
        self._check(self.lib.secpe_rotate_batch(self.h, n, cin, _p(st, C.c_int64), C.c_void_p(ws.data_ptr()),
                                                ws.numel() * 8, cout))
        for o, c in zip(outs, cout):
            o.level, o.scale = c.level, c.scale
        return outs

    # -- parity interfaces -------------------------------------------------------
    def export(self, ct):
        out = np.zeros((2, ct.level + 1, self.N), dtype=np.uint64)
        c = ct._c()
        self._check(self.lib.secpe_ct_export(self.h, C.byref(c), _p(out, C.c_uint64)))
        return out

    def import_(self, arr, scale):
        arr = np.ascontiguousarray(arr, dtype=np.uint64)
        ct = self.new_ct()
        c = ct._c()
        self._check(self.lib.secpe_ct_import(self.h, _p(arr, C.c_uint64), arr.shape[1] - 1, float(scale), C.byref(c)))
        ct.level, ct.scale = c.level, c.scale
        return ct

    def key_limb(self, key, digit, which, prime):
        out = np.zeros(self.N, dtype=np.uint64)
        self._check(self.lib.secpe_key_export(self.h, C.c_void_p(self.evk.data_ptr()), key, digit, which, prime,
                                              _p(out, C.c_uint64)))
        return out

    def secret(self):
        out = np.zeros(self.N, dtype=np.int64)
        self._check(self.lib.secpe_sk_export(self.h, C.c_void_p(self.sk.data_ptr()), _p(out, C.c_int64)))
        return out

    def _opws(self):
        if getattr(self, "_ows", None) is None:
            self._ows = self._empty(self.lib.secpe_op_workspace_bytes(self.h))
        return self._ows

    def _op(self, fn, *args, ws=True):
        out = self.new_ct()
        c = out._c()
        if ws:
            w = self._opws()
            self._check(fn(self.h, *args, C.c_void_p(w.data_ptr()), w.numel() * 8, C.byref(c)))
        else:
            self._check(fn(self.h, *args, C.byref(c)))
        out.level, out.scale = c.level, c.scale
        return out

    def add(self, a, b):
        return self._op(self.lib.secpe_op_add, C.byref(a._c()), C.byref(b._c()), ws=False)

    def sub(self, a, b):
        return self._op(self.lib.secpe_op_sub, C.byref(a._c()), C.byref(b._c()), ws=False)

    def add_const(self, a, v):
        return self._op(self.lib.secpe_op_add_const, C.byref(a._c()), float(v), ws=False)

    def mul_const(self, a, v, target):
        return self._op(self.lib.secpe_op_mul_const, C.byref(a._c()), float(v), float(target))

    def lincomb(self, a, va, b, vb, target, rescale=True):
        return self._op(self.lib.secpe_op_lincomb, C.byref(a._c()), float(va),
                        C.byref(b._c()) if b is not None else None, float(vb), float(target), int(bool(rescale)))

    def mul_plain(self, a, v, target):
        v = np.ascontiguousarray(v, dtype=np.float64)
        self._keep = v
        return self._op(self.lib.secpe_op_mul_plain, C.byref(a._c()), _p(v, C.c_double), len(v), float(target))

    def rescale(self, a):
        return self._op(self.lib.secpe_op_rescale, C.byref(a._c()))

    def mul_relin(self, a, b):
        return self._op(self.lib.secpe_op_mul_relin, C.byref(a._c()), C.byref(b._c()))

    def mul_relin_rescale(self, a, b):
        return self._op(self.lib.secpe_op_mul_relin_rescale, C.byref(a._c()), C.byref(b._c()))

    def rotate(self, a, step):
        return self._op(self.lib.secpe_op_rotate, C.byref(a._c()), int(step))

    def refresh(self, a, seed, index, owner):
        return self._op(self.lib.secpe_op_refresh, _owner(owner), C.byref(a._c()), int(seed), int(index))

    def eval_odd9(self, a, coef, gain, target):
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        self._keep = coef
        return self._op(self.lib.secpe_op_eval_odd9, C.byref(a._c()), _p(coef, C.c_double), float(gain), float(target))

    def key_switch(self, key, d):
        d = np.ascontiguousarray(d, dtype=np.uint64)
        level = d.shape[0] - 1
        u0 = np.zeros_like(d)
        u1 = np.zeros_like(d)
        w = self._opws()
        self._check(self.lib.secpe_op_key_switch(self.h, key, _p(d, C.c_uint64), level, C.c_void_p(w.data_ptr()),
                                                 w.numel() * 8, _p(u0, C.c_uint64), _p(u1, C.c_uint64)))
        return u0, u1

    def ntt(self, prime, limbs):
        limbs = np.ascontiguousarray(np.atleast_2d(limbs), dtype=np.uint64)
        fw = np.zeros_like(limbs)
        rt = np.zeros_like(limbs)
        self._check(self.lib.secpe_op_ntt(self.h, prime, _p(limbs, C.c_uint64), limbs.shape[0], _p(fw, C.c_uint64),
                                          _p(rt, C.c_uint64)))
        return fw, rt

    def ring_mul(self, prime, a, b):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.zeros(self.N, dtype=np.uint64)
        self._check(self.lib.secpe_op_ring_mul(self.h, prime, _p(a, C.c_uint64), _p(b, C.c_uint64),
                                               _p(out, C.c_uint64)))
        return out

    def encode(self, z, scale):
        z = np.ascontiguousarray(z, dtype=np.float64)
        out = np.zeros(self.N, dtype=np.int64)
        self._check(self.lib.secpe_op_encode(self.h, _p(z, C.c_double), len(z), float(scale), _p(out, C.c_int64)))
        return out


class Server:
    """Continuous-batching request loop over one workspace (secpe_server_*)."""

    def __init__(self, ctx, ws_bytes, max_active=256, owner=None):
        self.ctx = ctx
        self.lib = ctx.lib
        self.owner = owner
        self.ws = ctx._empty(ws_bytes)
        h = C.c_void_p()
        ctx._check(self.lib.secpe_server_create(ctx.h, _owner(owner), C.c_void_p(self.ws.data_ptr()),
                                                self.ws.numel() * 8, int(max_active), C.byref(h)))
        self.h = h
        self.results = {}
        self._inputs = {}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.secpe_server_destroy(self.h)
            self.h = None

    @property
    def in_flight(self):
        """Requests submitted and not yet reported complete."""
        return len(self._inputs)

    def request_bytes(self, K, Cc):
        return self.lib.secpe_server_request_bytes(self.ctx.h, int(K), int(Cc))

    def submit(self, ct, K, Cc, d_min, d_max, refresh_seed, out=None):
        out = out if out is not None else self.ctx.new_ct()
        t = C.c_uint64(0)
        c = ct._c()
        self.ctx._check(self.lib.secpe_server_submit(self.h, C.byref(c), int(K), int(Cc), float(d_min), float(d_max),
                                                     int(refresh_seed), C.c_void_p(out.buf.data_ptr()), C.byref(t)))
        self._inputs[t.value] = (ct, out)
        return t.value

    def step(self, cap=1024):
        """Launch and collect: (completed tickets, active, pending)."""
        return self._report(self.lib.secpe_server_step, cap)

    def launch(self):
        """Queue the next submission without waiting (pair with collect)."""
        self.ctx._check(self.lib.secpe_server_launch(self.h))

    def ready(self):
        """True when collect would not wait."""
        r = self.lib.secpe_server_ready(self.h)
        self.ctx._check(min(r, 0))
        return r == 1

    def collect(self, cap=1024):
        """Wait for the launched submission: (completed tickets, active, pending)."""
        return self._report(self.lib.secpe_server_collect, cap)

    def _report(self, fn, cap):
        n = C.c_int(0)
        na = C.c_int(0)
        npd = C.c_int(0)
        tk = np.zeros(cap, dtype=np.uint64)
        lv = np.zeros(cap, dtype=np.int32)
        sc = np.zeros(cap)
        self.ctx._check(fn(self.h, cap, C.byref(n), _p(tk, C.c_uint64), _p(lv, C.c_int), _p(sc, C.c_double),
                           C.byref(na), C.byref(npd)))
        done = []
        for i in range(n.value):
            t = int(tk[i])
            ct, out = self._inputs.pop(t)
            out.level, out.scale = int(lv[i]), float(sc[i])
            self.results[t] = out
            done.append(t)
        return done, na.value, npd.value
