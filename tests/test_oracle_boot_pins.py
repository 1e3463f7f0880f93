"""Pins of the oracle's bootstrapping against the mathematics it approximates.

The paper refreshes ciphertexts by bootstrapping (arXiv 2502.00847, Sec. 2.2;
Sec. 4.1) without giving its steps; the oracle follows the standard pipeline
(scale-down, ModRaise, CoeffToSlot, EvalMod, SlotToCoeff).  Each test checks one
step against its definition written here with numpy: the canonical embedding
as a dense matrix, Chebyshev interpolation through numpy's own routines, the
sine it approximates, and the identity the whole bootstrap must realise.
"""
import numpy as np
import pytest

import workload as W
from conftest import make_oracle
from oracle import sim
from oracle.ckks import argmax_rotation_steps

P = W.PARAMS["tiny_boot"]


def _embedding(o):
    """U_jk = zeta^(5^j k), j < N/2, k < N (slot j <-> root zeta^(5^j), zeta = e^(i pi / N))."""
    n, m2 = o.n, 2 * o.n
    g5 = np.array([pow(5, j, m2) for j in range(o.slots)], dtype=np.int64)
    k = np.arange(n, dtype=np.int64)
    return np.exp(1j * np.pi * ((g5[:, None] * k[None, :]) % m2) / n)


def _bitrev(S):
    L = S.bit_length() - 1
    return np.array([int(format(i, f"0{L}b")[::-1], 2) for i in range(S)])


def _cdecode(o, ct, E=None):
    """complex slot values of a ciphertext: decrypt to integers, evaluate at the roots"""
    E = _embedding(o) if E is None else E
    return E @ o.decrypt(ct).astype(np.float64) / ct.scale


@pytest.fixture(scope="module")
def boot():
    o = make_oracle("tiny_boot")
    steps = sorted(set(o.boot_steps()) | set(argmax_rotation_steps(4, 4, o.slots)))
    o.keygen(77, steps)
    return o, _embedding(o)


def test_bootstrap_level_budget():
    """2 * groups linear-transform levels, log2(deg+1) + 1 for the Chebyshev sum, r double angles."""
    o = make_oracle("tiny_boot")
    k = int(np.log2(P["boot_deg"] + 1))
    assert o.boot_out_level() == P["n_q"] - 1 - (2 * P["boot_groups"] + k + 1 + P["boot_r"])
    assert o.refresh_level == o.boot_out_level()
    # a chain too short for the pipeline is refused
    short = make_oracle("tiny_boot", n_q=12)
    assert short.boot_out_level() == -1


def test_sparse_secret_weight():
    """Each coefficient nonzero with probability h/N, values +-1."""
    o = make_oracle("tiny_boot")
    o.gen_secret(5)
    s = o.secret()
    assert set(np.unique(s)) <= {-1, 0, 1}
    w = int(np.count_nonzero(s))
    h = P["h"]
    assert abs(w - h) < 5 * np.sqrt(h)


def test_coeff_to_slot_is_inverse_embedding():
    """The CoeffToSlot groups, applied in order, equal P U^-1 / (2 (K+1)) where
    U_jk = zeta^(5^j k) on the N/2 complex coefficients t_k + i t_(k+N/2) and P
    the bit reversal (Cheon et al. 2018: the special FFT factorised)."""
    o = make_oracle("tiny_boot")
    S = o.slots
    E = _embedding(o)
    U = E[:, :S]
    rng = np.random.default_rng(1)
    z = rng.normal(size=S) + 1j * rng.normal(size=S)
    v = z
    for g in range(P["boot_groups"]):
        v = o.boot_group_apply(1, g, v)
    ref = np.linalg.solve(U, z)[_bitrev(S)] / (2 * (P["boot_K"] + 1))
    assert np.abs(v - ref).max() < 1e-12 * np.abs(ref).max() * S


def test_slot_to_coeff_is_embedding():
    """The SlotToCoeff groups equal U P^-1 times 2^ratio / (2 pi)."""
    o = make_oracle("tiny_boot")
    S = o.slots
    U = _embedding(o)[:, :S]
    rng = np.random.default_rng(2)
    w = rng.normal(size=S) + 1j * rng.normal(size=S)
    v = w
    for g in range(P["boot_groups"]):
        v = o.boot_group_apply(0, g, v)
    wn = np.empty_like(w)
    wn[_bitrev(S)] = w
    ref = U @ wn * 2.0 ** P["boot_ratio"] / (2 * np.pi)
    assert np.abs(v - ref).max() < 1e-12 * np.abs(ref).max() * S


def test_chebyshev_interpolant():
    """c_j interpolate f(u) = cos(2 pi ((K+1) u - 1/4) / 2^r) at the deg+1 Chebyshev
    nodes (numpy's chebval), and approximate it on the whole interval."""
    o = make_oracle("tiny_boot")
    K, r, deg = P["boot_K"], P["boot_r"], P["boot_deg"]
    c = o.boot_cheb()
    f = lambda u: np.cos(2 * np.pi * ((K + 1) * u - 0.25) / 2**r)
    n = deg + 1
    nodes = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    assert np.abs(np.polynomial.chebyshev.chebval(nodes, c) - f(nodes)).max() < 1e-13
    u = np.linspace(-1, 1, 4001)
    assert np.abs(np.polynomial.chebyshev.chebval(u, c) - f(u)).max() < 1e-9
    # composed with r double angles this is sin(2 pi x) on |x| <= K + 1
    y = np.polynomial.chebyshev.chebval(u, c)
    for _ in range(r):
        y = 2 * y * y - 1
    assert np.abs(y - np.sin(2 * np.pi * (K + 1) * u)).max() < 1e-8


def test_encode_complex_is_inverse_embedding():
    o = make_oracle("tiny_boot")
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, o.slots) + 1j * rng.uniform(-1, 1, o.slots)
    scale = 2.0**40
    m = o.encode_complex(z, scale)
    got = _embedding(o) @ m.astype(np.float64) / scale
    assert np.abs(got - z).max() < o.n / scale
    # real values encode as the real encoder does
    assert np.array_equal(o.encode_complex(z.real, scale), o.encode(z.real, scale))


def test_mod_raise_keeps_residue_mod_q0(boot):
    """After the scale-down to level 0 at T_b = q_0 2^-ratio and the lift, the
    message t satisfies t = m (mod q_0) with m encoding z at T_b, t - m = q_0 I,
    |I| <= K; limb 0 is unchanged."""
    o, E = boot
    q0 = int(o.primes[0])
    rng = np.random.default_rng(4)
    z = rng.uniform(-1, 1, o.slots)
    sc = 2.0**50
    ct = o.lower(o.encrypt(o.encode(z, sc), sc, 5), 1)
    tb = float(q0) * 2.0 ** -P["boot_ratio"]
    x0 = o.lincomb(ct, 1.0, None, 0.0, tb, 1)
    assert x0.level == 0 and x0.scale == tb
    r = o.mod_raise(x0)
    assert r.level == o.n_q - 1 and r.scale == float(q0)
    assert np.array_equal(r.export()[:, 0, :], x0.export()[:, 0, :])
    t = [int(v) for v in o.decrypt(r)]
    m = [((v + q0 // 2) % q0) - q0 // 2 for v in t]
    I = [(a - b) // q0 for a, b in zip(t, m)]
    assert all((a - b) % q0 == 0 for a, b in zip(t, m))
    assert max(abs(v) for v in I) <= P["boot_K"]
    zz = (E @ np.array(m, dtype=np.float64)).real / tb
    assert np.abs(zz - z).max() < 1e-6


def test_monomial_half_multiplies_slots_by_i(boot):
    """X^(N/2) evaluates to i at every root zeta^(5^j) (5^j = 1 mod 4)."""
    o, E = boot
    rng = np.random.default_rng(6)
    z = rng.uniform(-1, 1, o.slots)
    sc = 2.0**40
    ct = o.lower(o.encrypt(o.encode(z, sc), sc, 7), 3)
    a = _cdecode(o, o.mul_monomial_half(ct, 0), E)
    b = _cdecode(o, o.mul_monomial_half(ct, 1), E)
    assert np.abs(a - 1j * z).max() < 1e-6
    assert np.abs(b + 1j * z).max() < 1e-6


def test_eval_mod_is_sine(boot):
    """EvalMod on u = x / (K+1), x = I + eps near integers, returns sin(2 pi x)
    (Han-Ki 2020: the scaled cosine, then double angles), r + log2(deg+1) + 1 levels down."""
    o, _ = boot
    K = P["boot_K"]
    rng = np.random.default_rng(8)
    x = rng.integers(-K, K + 1, o.slots) + rng.uniform(-2.0**-8, 2.0**-8, o.slots)
    sc = 2.0**50
    lvl = o.n_q - 1 - P["boot_groups"]
    ct = o.lower(o.encrypt(o.encode(x / (K + 1), sc), sc, 9), lvl)
    y = o.eval_mod(ct)
    k = int(np.log2(P["boot_deg"] + 1))
    assert y.level == lvl - (k + 1 + P["boot_r"])
    assert abs(y.scale / sc - 1) < 1e-6  # the double angles leave Delta^2 / q per step
    got = o.decrypt_decode(y, o.slots)
    assert np.abs(got - np.sin(2 * np.pi * x)).max() < 1e-7


@pytest.mark.parametrize("kind,level", [("uniform", 1), ("sparse", 1), ("uniform", 7)])
def test_bootstrap_is_identity(boot, kind, level):
    """A bootstrapped ciphertext decrypts to its input (|z| <= 1) at the output
    level with scale Delta, within 2^-16 on N = 2^10."""
    o, _ = boot
    rng = np.random.default_rng(10 + level)
    if kind == "uniform":
        z = rng.uniform(-1, 1, o.slots)
    else:
        z = np.zeros(o.slots)
        z[:8] = rng.uniform(0, 1, 8)
    sc = 2.0**49
    ct = o.lower(o.encrypt(o.encode(z, sc), sc, 11), level)
    o.reset_counters()
    b = o.bootstrap(ct)
    assert b.level == o.boot_out_level()
    assert b.scale == 2.0 ** P["log_scale"]
    assert np.abs(o.decrypt_decode(b, o.slots) - z).max() < 2.0**-16
    assert o.counters()["refresh"] == 1


def test_argmax_with_bootstrapping(boot):
    """Algorithm 1 with every refresh a bootstrap: the index is the plaintext
    argmax and z follows the FP64 simulation of the same polynomials."""
    o, _ = boot
    K, C = 2, 4
    y = W.logits(9, 5, K, C)
    lo, hi = W.d_bounds(K)
    o.reset_counters()
    z = o.decrypt_decode(o.eval_argmax(o.encrypt_logits(y, 3), K, C, lo, hi, 4), C)
    cnt = o.counters()
    assert cnt["refresh"] >= 1 and cnt["sign"] == 3
    zs = sim.t1_argmax(y, lo, hi, o.slots)[:C]
    assert np.abs(z - zs).max() < 1e-3
    assert int(np.argmax(z)) == sim.t0_argmax(y)[0]


# ---------------------------------------------------------------------------
# sparse-slot bootstrapping: n slots kept, the n-slot special FFT
SPARSE_N = 32


def _embedding_n(n):
    """U'_jk = xi^(5^j k), j, k < n, xi = e^(i pi / 2n): the slots of a polynomial in
    Y = X^(N/2n) with coefficients t_k + i t_(k+n) (xi^n = i and 5^j = 1 mod 4)."""
    m4 = 4 * n
    g5 = np.array([pow(5, j, m4) for j in range(n)], dtype=np.int64)
    k = np.arange(n, dtype=np.int64)
    return np.exp(2j * np.pi * ((g5[:, None] * k[None, :]) % m4) / m4)


def test_sparse_transforms_are_the_n_slot_embedding():
    """On one 2n period of the slots: the sparse CoeffToSlot maps an n-periodic
    z to [P U'^-1 z (n / (N/2)) / (2 (K+1)), 0], and the sparse SlotToCoeff
    maps [a, b] to U' P^-1 (a + i b) 2^ratio / (2 pi), repeated with period n;
    U' is the n-slot embedding written here."""
    o = make_oracle("tiny_boot")
    n = SPARSE_N
    o.set_boot_sparse(n)
    U = _embedding_n(n)
    rng = np.random.default_rng(21)
    z = rng.normal(size=n) + 1j * rng.normal(size=n)
    v = o.boot_sparse_apply(1, np.tile(z, 2))
    ref = np.linalg.solve(U, z)[_bitrev(n)] / (2 * (P["boot_K"] + 1)) * n / o.slots
    assert np.abs(v[:n] - ref).max() < 1e-12 * np.abs(ref).max() * n
    assert np.abs(v[n:]).max() == 0.0
    a, b = rng.normal(size=n), rng.normal(size=n)
    w = o.boot_sparse_apply(0, np.concatenate([a, b]))
    zn = np.empty(n, dtype=complex)
    zn[_bitrev(n)] = a + 1j * b
    ref = U @ zn * 2.0 ** P["boot_ratio"] / (2 * np.pi)
    assert np.abs(w[:n] - ref).max() < 1e-12 * np.abs(ref).max() * n
    assert np.abs(w[n:] - ref).max() < 1e-12 * np.abs(ref).max() * n
    # U' is the embedding restricted to the subring: a polynomial in X^(N/2n)
    # has these slot values at the first n roots, repeated with period n
    E = _embedding(o)
    t = rng.normal(size=2 * n)
    poly = np.zeros(o.n)
    poly[:: o.n // (2 * n)] = t
    full = E @ poly
    assert np.abs(full[:n] - U @ (t[:n] + 1j * t[n:])).max() < 1e-9
    assert np.abs(full[n: 2 * n] - full[:n]).max() < 1e-9


@pytest.fixture(scope="module")
def sparse_boot():
    o = make_oracle("tiny_boot")
    o.set_boot_sparse(SPARSE_N)
    steps = sorted(set(o.boot_steps()) | set(argmax_rotation_steps(4, 4, o.slots)))
    o.keygen(77, steps)
    return o


def test_sparse_bootstrap_parameters_are_checked():
    o = make_oracle("tiny_boot")
    # a power of two, 2n <= N/2, at least one radix-2 stage per group
    for bad in [3, 24, 4, o.slots, 2 * o.slots]:
        with pytest.raises(ValueError):
            o.set_boot_sparse(bad)
    o.set_boot_sparse(8)
    # the trace steps n, 2n, ..., N/4 and RotR(n) are among the bootstrapping steps
    st = set(o.boot_steps())
    assert all(r in st for r in (8 << k for k in range(int(np.log2(o.slots // 8)))))
    assert o.slots - 8 in st


@pytest.mark.parametrize("kind", ["uniform", "few"])
def test_sparse_bootstrap_keeps_the_first_slots(sparse_boot, kind):
    """Slots [0, n) of the input come back, repeated with period n over all N/2
    slots, whatever the other slots held; same level and scale as the full
    pipeline, within 2^-16 on N = 2^10."""
    o = sparse_boot
    n = SPARSE_N
    rng = np.random.default_rng(31)
    z = rng.uniform(-1, 1, o.slots)
    if kind == "few":
        z[5:n] = 0.0
    sc = 2.0**49
    ct = o.lower(o.encrypt(o.encode(z, sc), sc, 13), 1)
    o.reset_counters()
    b = o.bootstrap_sparse(ct)
    assert b.level == o.boot_out_level() and b.scale == 2.0 ** P["log_scale"]
    got = o.decrypt_decode(b, o.slots)
    assert np.abs(got - np.tile(z[:n], o.slots // n)).max() < 2.0**-16
    cnt = o.counters()
    # two traces of log2(N/2n) rotations, conjugation, the join rotation, and the
    # linear transforms' baby and giant steps; EvalMod's products once, not twice
    assert cnt["refresh"] == 1
    assert cnt["rotate"] >= 2 * int(np.log2(o.slots // n)) + 2


def test_argmax_with_sparse_bootstrapping(sparse_boot):
    """Algorithm 1 (single query, C' = 4 so slots [0, 8) are live) with every
    refresh a sparse-slot bootstrap returns the plaintext argmax, and z follows
    the FP64 simulation."""
    o = sparse_boot
    K, C = 2, 4
    y = W.logits(9, 5, K, C)
    lo, hi = W.d_bounds(K)
    o.reset_counters()
    z = o.decrypt_decode(o.eval_argmax(o.encrypt_logits(y, 3), K, C, lo, hi, 4), C)
    cnt = o.counters()
    assert cnt["refresh"] >= 1 and cnt["sign"] == 3
    zs = sim.t1_argmax(y, lo, hi, o.slots)[:C]
    assert np.abs(z - zs).max() < 1e-3
    assert int(np.argmax(z)) == sim.t0_argmax(y)[0]


@pytest.mark.parametrize("k", [1, 3, 19])
def test_packed_bootstrap_returns_every_window(sparse_boot, k):
    """Window-packed refresh of k ciphertexts (W = n slots each, N/2W per full
    bootstrap): output j holds input j's slots [0, W) at [0, W), whatever the
    inputs held elsewhere, and in window i the window of input j + i of its
    group, cyclically within the group's N/2W windows (zero past its last
    input).  That is the packing sum_j RotR(v_j, jW) and the unpacking
    RotL(P', jW) written out; output level and scale as the full pipeline,
    within the full bootstrap's 2^-16 on N = 2^10."""
    o = sparse_boot
    W, S = SPARSE_N, o.slots
    per = S // W
    rng = np.random.default_rng(40 + k)
    zs, cts = [], []
    sc = 2.0**49
    for j in range(k):
        z = rng.uniform(-1, 1, S)
        zs.append(z)
        cts.append(o.lower(o.encrypt(o.encode(z, sc), sc, 100 + j), 1 + j % 3))
    o.reset_counters()
    outs = o.bootstrap_packed(cts)
    assert o.counters()["refresh"] == k
    for j, b in enumerate(outs):
        assert b.level == o.boot_out_level() and b.scale == 2.0 ** P["log_scale"]
        p0 = j - j % per
        m = min(per, k - p0)
        want = np.zeros(S)
        for i in range(per):
            src = (j - p0 + i) % per
            if src < m:
                want[i * W:(i + 1) * W] = zs[p0 + src][:W]
        got = o.decrypt_decode(b, S)
        assert np.abs(got - want).max() < 2.0**-16, j
