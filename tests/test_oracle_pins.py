"""Pins of the CPU oracle against mathematics it does not itself use.

Each test checks the oracle (tests/ may load it) against a closed form, an
invariant, brute force on tiny inputs, or a big-integer evaluation written
here in plain Python -- never against a retyped copy of the oracle's own
formula.  Citations are to arXiv 2502.00847.
"""
import itertools
import math

import numpy as np
import pytest

import workload as W
from conftest import make_oracle
from oracle import sim
from oracle.ckks import Oracle, argmax_rotation_steps, sign_coeffs


# ---------------------------------------------------------------- helpers ---
def _is_prime_trial(n):
    """Deterministic primality by Python big-int Miller-Rabin over the first 20 primes."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _crt(residues, moduli):
    """Centred big integer from residues (Python ints)."""
    Q = 1
    for q in moduli:
        Q *= q
    x = 0
    for r, q in zip(residues, moduli):
        Qi = Q // q
        x += int(r) * Qi * pow(Qi, -1, q)
    x %= Q
    return x - Q if x > Q // 2 else x


def _schoolbook_negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            v = int(a[i]) * int(b[j])
            if i + j < n:
                out[i + j] += v
            else:
                out[i + j - n] -= v
    return np.array([x % q for x in out], dtype=np.uint64)


def _dec_big(o, ct_arr, s, level):
    """Exact m = c0 + c1*s over Q_level, per coefficient, centred (big ints)."""
    primes = [int(p) for p in o.primes[: level + 1]]
    res = []
    for t, q in enumerate(primes):
        s_t = np.array([int(v) % q for v in s], dtype=np.uint64)
        c1s = o.ring_mul(t, ct_arr[1, t], s_t)
        res.append([(int(a) + int(b)) % q for a, b in zip(ct_arr[0, t], c1s)])
    return [_crt([res[t][i] for t in range(len(primes))], primes) for i in range(o.n)]


@pytest.fixture(scope="module")
def tiny():
    o = make_oracle("tiny")
    o.keygen(123, argmax_rotation_steps(8, 8, o.slots) + [3, 5])
    return o


# ----------------------------------------------------------------- primes ---
@pytest.mark.parametrize("name", ["toy", "tiny", "mini"])
def test_primes_rule(name):
    """RNS moduli (Sec. 2.2): distinct primes = 1 mod 2N; the chain alternates
    nearest-below / nearest-above 2^qbits, special primes are the largest below 2^pbits."""
    p = W.PARAMS[name]
    o = make_oracle(name)
    pr = [int(v) for v in o.primes]
    n2 = 2 << p["log_n"]
    assert len(set(pr)) == len(pr)
    for v in pr:
        assert v % n2 == 1 and _is_prime_trial(v)
    chain, special = pr[: p["n_q"]], pr[p["n_q"]:]
    base = 1 << p["q_bits"]
    below = [v for v in chain[0::2]]
    above = [v for v in chain[1::2]]
    assert all(v < base for v in below) and all(v > base for v in above)
    # nearest: no prime = 1 mod 2N lies between base and the chosen ones that was skipped
    cand_below = [c for c in range(base + 1 - n2, below[-1] - 1, -n2) if _is_prime_trial(c)]
    assert cand_below == below
    cand_above = [c for c in range(base + 1, above[-1] + 1, n2) if _is_prime_trial(c)]
    assert cand_above == above
    top = 1 << p["p_bits"]
    cand_sp = [c for c in range(top + 1 - n2, special[-1] - 1, -n2) if _is_prime_trial(c)]
    assert cand_sp == special
    assert max(pr) < 2**51


def test_psi_is_primitive_2n_root():
    o = make_oracle("tiny")
    for t, q in enumerate(int(v) for v in o.primes):
        psi = o.psi(t)
        assert pow(psi, o.n, q) == q - 1  # order exactly 2N


# -------------------------------------------------------------------- NTT ---
@pytest.mark.parametrize("log_n", [3, 4, 5, 7])
def test_ring_mul_matches_schoolbook(log_n):
    """Negacyclic product in Z_q[X]/(X^N+1) (Sec. 2.2) against the O(N^2) definition."""
    o = Oracle(log_n, 3, 30, 1, 51, 30)
    rng = np.random.default_rng(log_n)
    for t, q in enumerate(int(v) for v in o.primes):
        a = rng.integers(0, q, o.n, dtype=np.uint64)
        b = rng.integers(0, q, o.n, dtype=np.uint64)
        assert np.array_equal(o.ring_mul(t, a, b), _schoolbook_negacyclic(a, b, q))


def test_ring_mul_schoolbook_n1024():
    o = Oracle(10, 2, 40, 1, 51, 40)
    rng = np.random.default_rng(5)
    q = int(o.primes[1])
    a = rng.integers(0, q, o.n, dtype=np.uint64)
    b = rng.integers(-3, 4, o.n).astype(np.int64) % q
    b = b.astype(np.uint64)
    assert np.array_equal(o.ring_mul(1, a, b), _schoolbook_negacyclic(a, b, q))


def test_ntt_roundtrip_identity():
    o = make_oracle("toy")
    rng = np.random.default_rng(1)
    for t, q in enumerate(int(v) for v in o.primes):
        a = rng.integers(0, q, o.n, dtype=np.uint64)
        assert np.array_equal(o.ntt_roundtrip(t, a), a)


# --------------------------------------------------------------- encoding ---
def test_encode_matches_direct_root_evaluation():
    """Slot j holds m(zeta^(5^j))/scale, zeta = exp(i pi / N) (canonical embedding, Sec. 2.2)."""
    o = make_oracle("tiny")
    rng = np.random.default_rng(2)
    z = rng.uniform(-1, 1, o.slots)
    scale = 2.0**40
    m = o.encode(z, scale)
    k = np.arange(o.n)
    for j in [0, 1, 2, 17, o.slots - 1]:
        g = pow(5, j, 2 * o.n)
        val = np.sum(m.astype(np.float64) * np.exp(1j * np.pi * ((g * k) % (2 * o.n)) / o.n))
        assert abs(val.real / scale - z[j]) < 1e-9
        assert abs(val.imag / scale) < 1e-9
    # rounding: |m - scale * embed^-1(z)| <= 1/2, so decoding error <= N/(2 scale) per slot
    zz = o.decode(m, scale, 64)
    assert np.abs(zz - z[:64]).max() <= o.n / (2 * scale)


def test_automorphism_rotates_slots():
    """RotL(z, r) <-> X -> X^(5^r); index map X^i -> X^(i g mod 2N) with X^N = -1."""
    o = make_oracle("tiny")
    z = np.random.default_rng(3).uniform(-1, 1, o.slots)
    m = o.encode(z, 2.0**40)
    q = int(o.primes[0])
    for r in [1, 3, 100, o.slots - 1]:
        g = o.galois_elt(r)
        assert g == pow(5, r, 2 * o.n)
        a = (m % q).astype(np.uint64)
        out = o.automorph(0, a, g)
        ref = np.zeros(o.n, dtype=object)
        for i in range(o.n):
            j = (i * g) % (2 * o.n)
            if j < o.n:
                ref[j] = int(a[i])
            else:
                ref[j - o.n] = (q - int(a[i])) % q
        assert np.array_equal(out, ref.astype(np.uint64))
        cen = np.where(out > q // 2, out.astype(np.int64) - q, out.astype(np.int64))
        zz = o.decode(cen, 2.0**40, 16)
        assert np.abs(zz - np.roll(z, -r)[:16]).max() < 1e-8


# ---------------------------------------------------------- samplers/keys ---
def test_secret_is_ternary_and_balanced():
    o = make_oracle("toy")
    o.gen_secret(99)
    s = o.secret()
    assert set(np.unique(s)) <= {-1, 0, 1}
    counts = np.array([(s == v).sum() for v in (-1, 0, 1)]) / o.n
    assert np.all(np.abs(counts - 1 / 3) < 0.03)


def test_encrypt_decrypt_error_is_cbd21():
    """decrypt(encrypt(m)) = m + e exactly, e centred binomial with eta=21: |e| <= 21, var 10.5."""
    o = make_oracle("toy")
    o.keygen(5, [])
    rng = np.random.default_rng(4)
    m = rng.integers(-2**40, 2**40, o.n)
    ct = o.encrypt(m, 2.0**30, 77)
    e = o.decrypt(ct) - m
    assert np.abs(e).max() <= 21
    assert abs(e.mean()) < 0.2 and abs(e.var() - 10.5) < 0.8
    # c1 is uniform mod q: mean close to q/2
    arr = ct.export()
    for t, q in enumerate(int(v) for v in o.primes[: o.n_q]):
        assert arr[1, t].max() < q
        assert abs(arr[1, t].astype(np.float64).mean() / q - 0.5) < 0.02


def test_encrypt_is_deterministic_in_seed():
    o = make_oracle("tiny")
    o.keygen(5, [])
    m = np.arange(o.n, dtype=np.int64)
    a = o.encrypt(m, 2.0**40, 9).export()
    b = o.encrypt(m, 2.0**40, 9).export()
    c = o.encrypt(m, 2.0**40, 10).export()
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_switching_key_decrypts_to_gadget(tiny):
    """Each key digit satisfies b + a s = e + P T_j s' over QP with small e (the
    hybrid key-switching gadget); checked with big integers for the relin key."""
    o = tiny
    s = o.secret()
    pr = [int(v) for v in o.primes]
    n_q = o.n_q
    P = math.prod(pr[n_q:])
    # s' = s^2 over Z[X]/(X^N+1)
    s2 = np.zeros(o.n, dtype=object)
    nz = np.nonzero(s)[0]
    for i in nz:
        for j in nz:
            v = int(s[i]) * int(s[j])
            if i + j < o.n:
                s2[i + j] += v
            else:
                s2[i + j - o.n] -= v
    for j in range(o.dnum):
        for t, q in enumerate(pr):
            b = o.key_limb(0, j, 0, t)
            a = o.key_limb(0, j, 1, t)
            s_t = np.array([int(v) % q for v in s], dtype=np.uint64)
            as_ = o.ring_mul(t, a, s_t)
            in_digit = t < n_q and t // o.alpha == j
            for i in range(0, o.n, 61):
                e = (int(b[i]) + int(as_[i]) - (P * int(s2[i]) if in_digit else 0)) % q
                e = e - q if e > q // 2 else e
                assert abs(e) <= 21


# ---------------------------------------------------------- hom. operations -
def test_rescale_is_exact_rounding(tiny):
    """Rescale by q_l divides every coefficient of every polynomial by q_l with
    rounding to nearest: checked with big-integer CRT on the whole ciphertext."""
    o = tiny
    z = np.random.default_rng(6).uniform(-1, 1, o.slots)
    ct = o.encrypt(o.encode(z, 2.0**40), 2.0**40, 1)
    ct2 = o.mul_relin(ct, ct)
    a = ct2.export()
    b = o.rescale(ct2).export()
    pr = [int(v) for v in o.primes]
    lvl = a.shape[1] - 1
    ql = pr[lvl]
    for p in range(2):
        for i in range(0, o.n, 37):
            x = _crt([a[p, t, i] for t in range(lvl + 1)], pr[: lvl + 1])
            y = _crt([b[p, t, i] for t in range(lvl)], pr[:lvl])
            Qm = math.prod(pr[:lvl])
            r = x % ql
            r = r - ql if r > ql // 2 else r
            want = ((x - r) // ql) % Qm
            assert y % Qm == want


def test_homomorphic_ops_against_plaintext(tiny):
    o = tiny
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, o.slots)
    y = rng.uniform(-1, 1, o.slots)
    D = 2.0**40
    cx = o.encrypt(o.encode(x, D), D, 1)
    cy = o.encrypt(o.encode(y, D), D, 2)
    k = 32
    chk = lambda ct, ref, tol: np.abs(o.decrypt_decode(ct, k) - ref[:k]).max() < tol
    assert chk(o.add(cx, cy), x + y, 1e-8)
    assert chk(o.sub(cx, cy), x - y, 1e-8)
    assert chk(o.add_const(cx, 0.75), x + 0.75, 1e-8)
    mc = o.mul_const(cx, -3.25, D)
    assert mc.scale == D and chk(mc, -3.25 * x, 1e-8)
    v = rng.uniform(-1, 1, 16)
    mp = o.mul_plain(cx, v, D)
    ref = np.zeros(o.slots)
    ref[:16] = v * x[:16]
    assert chk(mp, ref, 1e-8)
    mr = o.mul_relin_rescale(cx, cy)
    assert mr.level == cx.level - 1 and chk(mr, x * y, 1e-7)
    for r in [1, 3, 5, 8, o.slots - 4]:
        assert chk(o.rotate(cx, r), np.roll(x, -r), 1e-7)


def _crt_pos(residues, moduli):
    Q = math.prod(moduli)
    x = 0
    for r, q in zip(residues, moduli):
        Qi = Q // q
        x += int(r) * Qi * pow(Qi, -1, q)
    return x % Q


def test_relin_rescale_is_floor_division(tiny):
    """Merged relinearise + rescale: with Y_w = P d_w + acc_w over Q_l u P (acc from
    ModUp + inner product), every output coefficient x satisfies
    |Y_w - B x| < (n_p + 1) B / 2 with B = P q_l, i.e. x = round(Y_w / B) + v,
    |v| <= (n_p + 1) / 2 (the centred approximate base conversion over the n_p + 1
    primes of B), checked with big integers."""
    o = tiny
    pr = [int(v) for v in o.primes]
    chain, special = pr[: o.n_q], pr[o.n_q:]
    P = math.prod(special)
    rng = np.random.default_rng(21)
    for level in (o.n_q - 1, 2):
        d = np.stack([np.stack([rng.integers(0, pr[t], o.n, dtype=np.uint64) for t in range(level + 1)])
                      for _ in range(3)])
        acc = o.key_switch_raw(0, d[2])
        out = o.relin_rescale3(d, 2.0**80).export()
        assert out.shape == (2, level, o.n)
        mods = chain[: level + 1] + special
        B = P * chain[level]
        Qm = math.prod(chain[:level])
        for w in range(2):
            for i in range(0, o.n, 29):
                y = [(P * int(d[w, t, i]) + int(acc[w][t, i])) % chain[t] for t in range(level + 1)]
                y += [int(acc[w][level + 1 + k, i]) for k in range(o.n_p)]
                Y = _crt_pos(y, mods)
                x = _crt_pos([out[w, t, i] for t in range(level)], chain[:level])
                r = (Y - B * x) % (Qm * B)
                r = r - Qm * B if r > Qm * B // 2 else r
                assert 2 * abs(r) < (o.n_p + 1) * B


def test_moddown_is_centred_division_by_p(tiny):
    """ModDown of the key-switch accumulator: every output coefficient u satisfies
    |A - P u| < n_p P / 2 for the big-integer accumulator A over Q_l u P (centred
    approximate conversion from the n_p special primes)."""
    o = tiny
    pr = [int(v) for v in o.primes]
    chain, special = pr[: o.n_q], pr[o.n_q:]
    P = math.prod(special)
    rng = np.random.default_rng(24)
    level = 3
    d = np.stack([rng.integers(0, pr[t], o.n, dtype=np.uint64) for t in range(level + 1)])
    acc = o.key_switch_raw(0, d)
    u = o.key_switch(0, d)
    Qm = math.prod(chain[: level + 1])
    mods = chain[: level + 1] + special
    for w in range(2):
        for i in range(0, o.n, 31):
            A = _crt_pos([int(acc[w][e, i]) for e in range(level + 1 + o.n_p)], mods)
            x = _crt_pos([int(u[w][t, i]) for t in range(level + 1)], chain[: level + 1])
            r = (A - P * x) % (Qm * P)
            r = r - Qm * P if r > Qm * P // 2 else r
            assert 2 * abs(r) < o.n_p * P


def test_relin_rescale_decrypts_to_quotient(tiny):
    """(out0 + out1 s) = (d0 + d1 s + d2 s^2) / q_l up to a small error, for
    uniformly random degree-2 inputs (big-integer decryption on both sides)."""
    o = tiny
    s = o.secret()
    pr = [int(v) for v in o.primes]
    rng = np.random.default_rng(22)
    level = 4
    d = np.stack([np.stack([rng.integers(0, pr[t], o.n, dtype=np.uint64) for t in range(level + 1)])
                  for _ in range(3)])
    out = o.relin_rescale3(d, 2.0**80).export()
    res = []
    for t in range(level + 1):
        q = pr[t]
        s_t = np.array([int(v) % q for v in s], dtype=np.uint64)
        s2 = o.ring_mul(t, s_t, s_t)
        m = (d[0, t].astype(object) + o.ring_mul(t, d[1, t], s_t).astype(object)
             + o.ring_mul(t, d[2, t], s2).astype(object)) % q
        res.append(m)
    got = _dec_big(o, out, s, level - 1)
    ql = pr[level]
    Qm = math.prod(pr[:level])
    for i in range(0, o.n, 17):
        m = _crt([res[t][i] for t in range(level + 1)], pr[: level + 1])
        e = (got[i] - (2 * m + ql) // (2 * ql)) % Qm
        e = e - Qm if e > Qm // 2 else e
        assert abs(e) < 2**14


def test_lincomb_values_and_scale(tiny):
    """K_a a + K_b b at an exact target scale, with and without the rescale."""
    o = tiny
    rng = np.random.default_rng(23)
    x = rng.uniform(-1, 1, o.slots)
    y = rng.uniform(-1, 1, o.slots)
    D = 2.0**40
    cx = o.encrypt(o.encode(x, D), D, 3)
    cy = o.encrypt(o.encode(y, D * 1.001), D * 1.001, 4)
    k = 32
    r = o.lincomb(cx, 0.7, cy, -1.3, D, True)
    assert r.level == cx.level - 1 and r.scale == D
    assert np.abs(o.decrypt_decode(r, k) - (0.7 * x[:k] - 1.3 * y[:k])).max() < 1e-8
    T = D * float(o.primes[cx.level - 1])
    u = o.lincomb(o.lower(cx, cx.level - 1), 0.25, None, 0.0, T, False)
    assert u.level == cx.level - 1 and u.scale == T
    assert np.abs(o.decrypt_decode(u, k) - 0.25 * x[:k]).max() < 1e-8


def test_key_switch_error_bound(tiny):
    """u0 + u1 s - d s' is small (hybrid key switching), for the relin key at two levels."""
    o = tiny
    s = o.secret()
    pr = [int(v) for v in o.primes]
    rng = np.random.default_rng(8)
    for level in [o.n_q - 1, 3]:
        d = np.stack([rng.integers(0, pr[t], o.n, dtype=np.uint64) for t in range(level + 1)])
        u0, u1 = o.key_switch(0, d)
        for t in range(level + 1):
            q = pr[t]
            s_t = np.array([int(v) % q for v in s], dtype=np.uint64)
            s2 = o.ring_mul(t, s_t, s_t)
            lhs = (u0[t].astype(object) + o.ring_mul(t, u1[t], s_t).astype(object)) % q
            rhs = o.ring_mul(t, d[t], s2).astype(object)
            e = (lhs - rhs) % q
            e = np.where(e > q // 2, e - q, e)
            assert np.abs(e.astype(np.float64)).max() < 2**20


def test_hoisted_rotation_decrypts_to_automorphism(tiny):
    """Hoisted rotations (one ModUp of c1, then X -> X^g on every raised digit
    before each inner product) decrypt to sigma_g(m) plus a key-switch error:
    exact big-integer decryption against an automorphism written here, for
    several steps sharing one ModUp, at the top level and at level 2.  Step 0
    is a copy; the regular RotL lands within the same bound."""
    o = tiny
    s = o.secret()
    D = 2.0**40
    x = np.random.default_rng(11).uniform(-1, 1, o.slots)
    steps = [0, 1, 3, 5, o.slots - 1]
    n = o.n

    def sigma(m, g):
        out = [0] * n
        for i, v in enumerate(m):
            j = (i * g) % (2 * n)
            if j < n:
                out[j] = v
            else:
                out[j - n] = -v
        return out

    for level in [o.n_q - 1, 2]:
        ct = o.lower(o.encrypt(o.encode(x, D), D, 5), level)
        m = _dec_big(o, ct.export(), s, level)
        outs = o.rotate_hoisted(ct, steps)
        assert len(outs) == len(steps)
        for st, r in zip(steps, outs):
            assert r.level == level and r.scale == ct.scale
            if st == 0:
                assert np.array_equal(r.export(), ct.export())
                continue
            want = sigma(m, o.galois_elt(st))
            got = _dec_big(o, r.export(), s, level)
            assert max(abs(a - b) for a, b in zip(got, want)) < 2**20
            reg = _dec_big(o, o.rotate(ct, st).export(), s, level)
            assert max(abs(a - b) for a, b in zip(reg, want)) < 2**20
            assert np.abs(o.decrypt_decode(r, 16) - np.roll(x, -st)[:16]).max() < 1e-8


def test_refresh_preserves_message(tiny):
    """The refresh stand-in re-encrypts the exact message: decryptions differ by a fresh e, |e| <= 21."""
    o = tiny
    z = np.random.default_rng(9).uniform(-1, 1, o.slots)
    ct = o.lower(o.encrypt(o.encode(z, 2.0**40), 2.0**40, 3), 2)
    rf = o.refresh(ct, 44, 0)
    assert rf.level == o.n_q - 1 and rf.scale == ct.scale
    assert np.abs(o.decrypt(rf) - o.decrypt(ct)).max() <= 21


def test_refresh_below_the_top_level():
    """With refresh_level = 6 the stand-in re-encrypts at level 6: same message (up to a
    fresh e), and its limbs are the first seven limbs of the top-level re-encryption
    (the randomness is per limb and per coefficient, independent of the level)."""
    o5 = make_oracle("tiny_r6")
    ot = make_oracle("tiny")
    for o in (o5, ot):
        o.keygen(123, [1])
    z = np.random.default_rng(10).uniform(-1, 1, o5.slots)
    ct5 = o5.lower(o5.encrypt(o5.encode(z, 2.0**40), 2.0**40, 3), 2)
    ctt = ot.lower(ot.encrypt(ot.encode(z, 2.0**40), 2.0**40, 3), 2)
    r5, rt = o5.refresh(ct5, 44, 1), ot.refresh(ctt, 44, 1)
    assert r5.level == 6 and rt.level == ot.n_q - 1
    assert np.abs(o5.decrypt(r5) - o5.decrypt(ct5)).max() <= 21
    assert np.array_equal(r5.export(), rt.export()[:, :7])


def test_argmax_with_low_refresh_level():
    """Algorithm 1 end to end with refreshes at level 6 (one Sign polynomial per
    refresh): the decrypted index equals the plaintext argmax."""
    o = make_oracle("tiny_r6")
    o.keygen(5, argmax_rotation_steps(8, 8, o.slots))
    for q, (K, C) in enumerate([(3, 5), (4, 3)]):
        y = W.logits(9, 100 + q, K, C)
        dmin, dmax = W.d_bounds(K)
        o.reset_counters()
        z = o.decrypt_decode(o.eval_argmax(o.encrypt_logits(y, 7 + q), K, C, dmin, dmax, 11 + q), C)
        i0, _, margin = sim.t0_argmax(y)
        if margin / (dmax - dmin) >= 2.0**-10:
            assert sim.decoded_index(z) == i0
        assert o.counters()["refresh"] >= 1


# ---------------------------------------------------------- Sign polynomials -
def test_f4_is_closed_form():
    """f_4 = sum_{i<=4} C(2i,i) 4^-i x (1-x^2)^i: expand with numpy polynomial algebra."""
    f, g = sign_coeffs()
    acc = np.polynomial.Polynomial([0.0])
    X = np.polynomial.Polynomial([0.0, 1.0])
    for i in range(5):
        acc = acc + math.comb(2 * i, i) / 4**i * X * (1 - X**2) ** i
    c = acc.coef
    assert np.allclose(c[1::2], f, atol=1e-15) and np.allclose(c[0::2], 0)
    # derivative is (315/128)(1-x^2)^4 and f(1) = 1
    d = acc.deriv()
    xs = np.linspace(-1, 1, 101)
    assert np.allclose(d(xs), 315 / 128 * (1 - xs**2) ** 4)
    assert abs(acc(1.0) - 1.0) < 1e-15
    assert np.allclose(f, sim.F4) and np.allclose(g, sim.G4)


def test_g4_properties():
    """g_4: odd, maps [-1,1] into [-1,1], positive on (0,1], slope 5850/1024 at 0."""
    xs = np.linspace(0, 1, 100001)[1:]
    gv = sim.odd_poly(sim.G4, xs)
    assert np.all(gv > 0) and np.all(gv <= 1.0)
    assert abs((sim.odd_poly(sim.G4, 1e-7) / 1e-7) - 5850 / 1024) < 1e-6
    assert np.allclose(sim.odd_poly(sim.G4, -xs), -gv)


def test_composite_sign_precision_reading():
    """Eq. 4 with d_f = d_g = 2: the 1e-4 band is reached only for |x| >= 2^-6, not
    2^-12 as the paper states (Sec. 3.2); (4,3) reaches 2^-12.3.  Also, no polynomial
    of degree 9^4 can reach 1e-4 at 2^-12 at all, so the reading is forced."""
    e22 = sim.sign_threshold(2, 2)
    assert -6.1 < e22 < -5.9
    e43 = sim.sign_threshold(4, 3)
    assert -12.4 < e43 < -12.2
    assert abs(sim.sign_composite(2.0**-12) - 0.048) < 0.002
    xs = np.linspace(-1, 1, 20001)
    assert np.abs(sim.sign_composite(xs)).max() <= 1.0 + 1e-12


def test_homomorphic_odd9_matches_fp64(tiny):
    o = tiny
    f, g = sign_coeffs()
    x = np.random.default_rng(10).uniform(-1, 1, o.slots)
    D = 2.0**40
    cx = o.encrypt(o.encode(x, D), D, 5)
    for coef in (f, g):
        p = o.eval_odd9(cx, coef, 1.0, D)
        assert p.level == cx.level - 4
        assert abs(p.scale / D - 1) < 1e-12
        assert np.abs(o.decrypt_decode(p, 32) - sim.odd_poly(coef, x[:32])).max() < 1e-6


# -------------------------------------------------------------- Algorithm 1 -
@pytest.mark.parametrize("C", [2, 3, 4, 5, 6])
def test_t1_exact_sign_gives_one_hot_brute_force(C):
    """With the exact sign, Algorithm 1 returns e_idx for every ordering of distinct inputs."""
    base = np.linspace(-1, 1, C) * 0.8
    for perm in itertools.permutations(range(C)):
        y = base[list(perm)][None, :]
        z = sim.t1_argmax(y, -6.0, 6.0, 64, exact_sign=True)
        # z = Sign(y - ymax) + 1: 1 at the max (Sign(0) = 0) and 0 elsewhere
        want = np.zeros(C)
        want[int(np.argmax(y[0]))] = 1.0
        assert np.array_equal(z, want)


def test_t1_max_and_quickmax_reduce_to_textbook():
    rng = np.random.default_rng(11)
    for _ in range(20):
        C = int(rng.integers(2, 20))
        K = int(rng.integers(1, 9))
        y = rng.standard_normal((K, C))
        z, aux = sim.t1_argmax(y, -6 * K, 6 * K, 256, exact_sign=True, return_all=True)
        ys = (y.sum(0) + 6 * K) / (12 * K)
        assert np.allclose(aux["ymax"][0], ys.max())
        assert np.allclose(aux["y"][:C], ys)


def test_t1_polynomial_index_matches_t0():
    for q in range(40):
        d = W.query(3, q)
        z = sim.t1_argmax(d["logits"], d["d_min"], d["d_max"], 1024)
        idx0, _, margin = sim.t0_argmax(d["logits"])
        if margin / (d["d_max"] - d["d_min"]) >= 2.0**-10:
            assert sim.decoded_index(z) == idx0


def test_counts_match_paper():
    """#Sign = log2 n + 1 and #rotations in Algorithm 1 = log2 n + 1 (Sec. 4.5), plus log2 K'
    rotations for the prompt sum."""
    o = make_oracle("tiny")
    o.keygen(1, argmax_rotation_steps(8, 8, o.slots))
    for K, C in [(2, 2), (3, 4), (4, 3)]:
        o.reset_counters()
        y = W.logits(9, K * 10 + C, K, C)
        dmin, dmax = W.d_bounds(K)
        o.eval_argmax(o.encrypt_logits(y, 1), K, C, dmin, dmax, 2)
        cnt = o.counters()
        lc = (C - 1).bit_length()
        lk = (K - 1).bit_length()
        assert cnt["sign"] == lc + 1
        assert cnt["rotate"] == lk + 1 + lc
        assert cnt["max"] == lc
        # four degree-9 polynomials of five relinearisations each per Sign, one per Max
        assert cnt["relin"] == 20 * (lc + 1) + lc


def _packed_group(seed, shapes):
    out = []
    for i, (K, C) in enumerate(shapes):
        y = W.logits(9, seed * 100 + i, K, C)
        lo, hi = W.d_bounds(K)
        out.append((y, lo, hi))
    return out


def test_t1_packed_blocks_do_not_interact():
    """Packed Algorithm 1 with the exact sign: every block's z is one-hot at its own
    plaintext argmax (no leakage between blocks), and a single block equals the
    unpacked Algorithm 1 bit for bit."""
    # integer logits and bounds +-64 keep every step exact in FP64 (dyadic values)
    rng = np.random.default_rng(31)
    for trial in range(40):
        n = int(rng.integers(1, 9))
        shapes = [(int(rng.integers(1, 9)), int(rng.integers(1, 9))) for _ in range(n)]
        blocks = [(rng.integers(-6, 7, size=sh).astype(np.float64), -64.0, 64.0) for sh in shapes]
        zs = sim.t1_argmax_packed(blocks, 512, exact_sign=True)
        for (y, lo, hi), z in zip(blocks, zs):
            tot = np.sum(y, 0)
            assert np.array_equal(z, (tot == tot.max()).astype(np.float64))
    y, lo, hi = _packed_group(99, [(3, 5)])[0]
    Kp, Cp, B = sim.packed_shape([(3, 5)])
    z1 = sim.t1_argmax_packed([(y, lo, hi)], 512)[0]
    assert np.array_equal(z1, sim.t1_argmax(y, lo, hi, 512))


def test_oracle_packed_argmax_tiny():
    """Encrypted packed Argmax (tiny parameters, four queries of uneven shape in one
    ciphertext): each block decrypts to the packed FP64 Algorithm 1 and to the plaintext
    argmax; the operation counts are those of one query of the group's padded shape."""
    o = make_oracle("tiny")
    o.keygen(5, argmax_rotation_steps(8, 8, o.slots))
    shapes = [(3, 5), (2, 3), (4, 2), (1, 4)]
    blocks = _packed_group(7, shapes)
    nb, kp, cp, bsz = o.packed_shape(shapes)
    assert (kp, cp, bsz) == (4, 8, 32) and nb == o.slots // 32
    ct = o.encrypt_packed([b[0] for b in blocks], 21)
    o.reset_counters()
    z = o.eval_argmax_packed(ct, shapes, [b[1] for b in blocks], [b[2] for b in blocks], 22)
    cnt = o.counters()
    assert cnt["sign"] == 3 + 1 and cnt["rotate"] == 2 + 1 + 3 and cnt["max"] == 3
    zs = o.decrypt_packed(z, shapes)
    ts = sim.t1_argmax_packed(blocks, o.slots)
    for (y, lo, hi), zb, tb in zip(blocks, zs, ts):
        assert np.abs(zb - tb).max() < 1e-3
        i0, _, margin = sim.t0_argmax(y)
        if margin / (hi - lo) >= 2.0**-10:
            assert sim.decoded_index(zb) == i0


def test_oracle_argmax_precise_sign_small_margins():
    """(d_g, d_f) = (4, 3): the encrypted Argmax (tiny parameters) decrypts to the
    plaintext argmax at normalised margins down to 2^-12, where (2, 2) is not
    guaranteed (its index threshold is 2^-10)."""
    o = make_oracle("tiny", dg=4, df=3)
    o.keygen(5, argmax_rotation_steps(4, 4, o.slots))
    rng = np.random.default_rng(41)
    K, C = 2, 4
    lo, hi = W.d_bounds(K)
    for trial in range(3):
        y = rng.uniform(-3, 3, (K, C))
        tot = y.sum(0)
        top = int(np.argmax(tot))
        # place the runner-up at normalised margin 2^-11.5 below the top
        second = (top + 1) % C
        y[0, second] += (tot[top] - 2.0**-11.5 * (hi - lo)) - tot[second]
        assert sim.t0_argmax(y)[0] == top
        z = o.decrypt_decode(o.eval_argmax(o.encrypt_logits(y, 3 + trial), K, C, lo, hi, 9 + trial), C)
        assert sim.decoded_index(z) == top


def test_t1_phoenix_exact_sign_is_one_hot():
    """The comparison path with the exact sign: the largest class wins all C-1
    comparisons, so z is e_idx (distinct dyadic inputs keep FP64 exact)."""
    rng = np.random.default_rng(51)
    for trial in range(30):
        K, C = int(rng.integers(1, 5)), int(rng.integers(2, 10))
        y = rng.permutation(np.arange(C) - C // 2)[None, :].repeat(K, 0).astype(np.float64) / 4
        z = sim.t1_argmax_phoenix(y, -64.0, 64.0, 256, exact_sign=True)
        want = np.zeros(C)
        want[int(np.argmax(y.sum(0)))] = 1.0
        assert np.array_equal(z, want)


def test_oracle_phoenix_argmax_tiny():
    """Encrypted comparison path (tiny parameters): decrypts to its FP64 simulation and
    the plaintext argmax, with the paper's counts: C Signs, C rotations after the
    prompt sum (Sec. 4.5)."""
    o = make_oracle("tiny")
    K, C = 2, 5
    lk = (K - 1).bit_length()
    steps = sorted(set(argmax_rotation_steps(K, C, o.slots) + list(range(1, C)) + [o.slots - C]))
    o.keygen(5, steps)
    y = W.logits(9, 700, K, C)
    lo, hi = W.d_bounds(K)
    ct = o.encrypt_logits(y, 31)
    o.reset_counters()
    z = o.decrypt_decode(o.eval_argmax_phoenix(ct, K, C, lo, hi, 32), C)
    cnt = o.counters()
    assert cnt["sign"] == C and cnt["rotate"] == lk + C
    t = sim.t1_argmax_phoenix(y, lo, hi, o.slots)
    assert np.abs(z - t).max() < 1e-3
    i0, _, margin = sim.t0_argmax(y)
    if margin / (hi - lo) >= 2.0**-8:
        assert sim.decoded_index(z) == i0


def test_packing_count_matches_paper():
    """2n slots per Argmax of length n -> N/(2n) inputs per ciphertext: 32768 slots, n=256 -> 64 (Sec. 3.2)."""
    o_slots = (1 << W.PARAMS["full"]["log_n"]) // 2
    assert o_slots == 32768 and o_slots // (2 * 256) == 64


def test_oracle_argmax_toy_end_to_end():
    """Toy parameters (N=2^13, 8 x 30-bit primes, scale 2^30), K=4, C=2: index equals T0,
    z within 1e-2 of the FP64 Algorithm 1 (T1)."""
    o = make_oracle("toy")
    o.keygen(W.KEYGEN_SEED, argmax_rotation_steps(4, 2, o.slots))
    d = W.query(1, 0)
    ct = o.encrypt_logits(d["logits"], d["encrypt_seed"])
    z = o.decrypt_decode(o.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"]), d["C"])
    t1 = sim.t1_argmax(d["logits"], d["d_min"], d["d_max"], o.slots)
    assert sim.decoded_index(z) == sim.t0_argmax(d["logits"])[0]
    assert np.abs(z - t1).max() < 1e-2
