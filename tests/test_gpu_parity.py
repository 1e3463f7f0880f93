"""GPU parity: every step of the HIP path is bit-exact with the CPU oracle on the
same seeded inputs (coefficient-domain residues compared element by element),
through the C ABI (include/secpe.h) via its Python binding.

Parameter sets: 'tiny' (N=2^10, single-pass NTT), 'p11' and 'p12' (the other
single-pass sizes), 'p13' (N=2^13, the toy's two-pass NTT split 2^6 x 2^7),
'p14' (2^7 x 2^7), 'p15' (2^7 x 2^8).  Full N=2^16 lives in test_gpu_full.py.
"""
import numpy as np
import pytest

import workload as W
from oracle import sim
from oracle.ckks import Oracle, sign_coeffs

pytestmark = pytest.mark.gpu

SEED = 0xC0FFEE
EXTRA_STEPS = [3, 5]


def _params(name):
    if name == "p13":
        return dict(log_n=13, n_q=8, q_bits=36, n_p=2, p_bits=51, log_scale=36, dg=2, df=2, min_level=1)
    if name == "tiny43":
        return dict(W.PARAMS["tiny"], dg=4, df=3)
    if name == "tiny52":
        return dict(W.PARAMS["tiny"], dg=5, df=2)
    if name == "p13_r6":
        return dict(_params("p13"), refresh_level=6)
    if name == "p14":
        return dict(log_n=14, n_q=8, q_bits=40, n_p=3, p_bits=51, log_scale=40, dg=2, df=2, min_level=1)
    if name == "p15":
        return dict(log_n=15, n_q=8, q_bits=40, n_p=3, p_bits=51, log_scale=40, dg=2, df=2, min_level=1)
    if name in ("p11", "p12"):
        return dict(log_n=int(name[1:]), n_q=8, q_bits=40, n_p=3, p_bits=51, log_scale=40, dg=2, df=2, min_level=1)
    return dict(W.PARAMS[name])


def _pair(name, k_max=8, c_max=8):
    from paper_2502_00847_amd.secpe import Context
    p = _params(name)
    g = Context(p)
    o = Oracle.from_params(p)
    steps = g.argmax_steps(k_max, c_max) + EXTRA_STEPS
    print(f"[pair] {name} keygen {len(steps)} rotation keys", flush=True)
    g.keygen(SEED, steps)
    g.owner = g.key_owner()
    o.keygen(SEED, steps)
    return g, o, steps


@pytest.fixture(scope="module")
def tiny():
    return _pair("tiny")


@pytest.fixture(scope="module")
def p13():
    return _pair("p13", 4, 4)


def _rand_ct(o, seed, scale=None, level=None):
    scale = scale or 2.0 ** o.log_scale
    z = np.random.default_rng(seed).uniform(-1, 1, o.slots)
    ct = o.encrypt(o.encode(z, scale), scale, seed)
    if level is not None:
        ct = o.lower(ct, level)
    return ct, z


def _same(g, gct, oct_):
    assert gct.level == oct_.level, (gct.level, oct_.level)
    assert gct.scale == oct_.scale, (gct.scale, oct_.scale)
    a = g.export(gct)
    b = oct_.export()
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        raise AssertionError(f"{len(bad)} residues differ, first at {bad[:5].tolist()}")


def test_library_exports_every_declared_symbol():
    from paper_2502_00847_amd import secpe
    lib = secpe.load()
    for name in secpe.exported_symbols():
        assert hasattr(lib, name)


@pytest.mark.parametrize("name", ["tiny", "p13", "p14", "full"])
def test_primes_match_oracle(name):
    from paper_2502_00847_amd.secpe import Context
    p = _params(name)
    g = Context(p)
    o = Oracle.from_params(p)
    assert np.array_equal(g.primes, o.primes)


@pytest.mark.parametrize("name", ["tiny", "p13", "p14", "full"])
def test_ntt_roundtrip_and_negacyclic_product(name):
    """NTT then inverse NTT is the identity; pointwise product in the NTT domain
    equals the oracle's negacyclic product (itself pinned to schoolbook)."""
    from paper_2502_00847_amd.secpe import Context
    p = _params(name)
    g = Context(p)
    o = Oracle.from_params(p)
    rng = np.random.default_rng(1)
    primes = [int(v) for v in g.primes]
    for t in [0, 1, len(primes) - 1]:
        q = primes[t]
        a = rng.integers(0, q, (3, g.N), dtype=np.uint64)
        fw, rt = g.ntt(t, a)
        assert np.array_equal(rt, a)
        assert fw.max() < q
        b = rng.integers(0, q, g.N, dtype=np.uint64)
        assert np.array_equal(g.ring_mul(t, a[0], b), o.ring_mul(t, a[0], b))


def test_ntt_edge_values():
    """All-zero, all-(q-1) and a unit vector survive the round trip; X * X^(N-1) = -1."""
    from paper_2502_00847_amd.secpe import Context
    p = _params("p14")
    g = Context(p)
    q = int(g.primes[2])
    for v in (np.zeros(g.N), np.full(g.N, q - 1), np.eye(1, g.N, 7)[0]):
        v = v.astype(np.uint64)
        assert np.array_equal(g.ntt(2, v)[1][0], v)
    x = np.zeros(g.N, dtype=np.uint64)
    x[1] = 1
    y = np.zeros(g.N, dtype=np.uint64)
    y[g.N - 1] = 1
    r = g.ring_mul(2, x, y)
    want = np.zeros(g.N, dtype=np.uint64)
    want[0] = q - 1
    assert np.array_equal(r, want)


@pytest.mark.parametrize("nslots", [1, 7, 64, 512])
def test_encode_matches_oracle(tiny, nslots):
    g, o, _ = tiny
    rng = np.random.default_rng(nslots)
    for scale in (2.0**40, 2.0**40 * 1.0000123, 12345.678):
        z = rng.uniform(-6, 6, nslots)
        assert np.array_equal(g.encode(z, scale), o.encode(z, scale))


def test_secret_and_switching_keys_match(tiny):
    g, o, steps = tiny
    assert np.array_equal(g.secret(), o.secret())
    n_mod = o.n_q + o.n_p
    for key, gal in [(0, 0), (1, o.galois_elt(steps[0])), (len(steps), o.galois_elt(steps[-1]))]:
        for digit in range(o.dnum):
            for which in (0, 1):
                for t in (0, o.n_q - 1, n_mod - 1):
                    assert np.array_equal(g.key_limb(key, digit, which, t), o.key_limb(gal, digit, which, t))


def test_encrypt_bit_exact(tiny):
    g, o, _ = tiny
    d = W.query(3, 5)
    _same(g, g.encrypt(d["logits"], d["encrypt_seed"]), o.encrypt_logits(d["logits"], d["encrypt_seed"]))
    m = np.random.default_rng(3).integers(-2**45, 2**45, g.N)
    _same(g, g.encrypt_coeffs(m, 2.0**40, 99), o.encrypt(m, 2.0**40, 99))


def test_decrypt_matches(tiny):
    g, o, _ = tiny
    ct, z = _rand_ct(o, 4)
    gct = g.import_(ct.export(), ct.scale)
    assert np.array_equal(g.decrypt_coeffs(gct), o.decrypt(ct))
    zz, idx = g.decrypt(gct, 16)
    assert np.allclose(zz, o.decrypt_decode(ct, 16), rtol=0, atol=1e-12)
    assert idx == int(np.argmax(zz))


def test_import_export_roundtrip(tiny):
    g, o, _ = tiny
    ct, _ = _rand_ct(o, 5, level=3)
    arr = ct.export()
    assert np.array_equal(g.export(g.import_(arr, ct.scale)), arr)


def test_elementwise_ops_bit_exact(tiny):
    g, o, _ = tiny
    a, _ = _rand_ct(o, 6)
    b, _ = _rand_ct(o, 7)
    bl = o.lower(b, 4)
    ga, gb, gbl = (g.import_(c.export(), c.scale) for c in (a, b, bl))
    _same(g, g.add(ga, gb), o.add(a, b))
    _same(g, g.sub(ga, gbl), o.sub(a, bl))
    _same(g, g.add_const(ga, -0.3125), o.add_const(a, -0.3125))
    _same(g, g.mul_const(ga, 3.7, 2.0**40 * 1.001), o.mul_const(a, 3.7, 2.0**40 * 1.001))
    _same(g, g.mul_const(gbl, -113.25, 2.0**39), o.mul_const(bl, -113.25, 2.0**39))
    v = np.random.default_rng(8).uniform(-1, 1, 13)
    _same(g, g.mul_plain(ga, v, 2.0**40), o.mul_plain(a, v, 2.0**40))
    _same(g, g.rescale(ga), o.rescale(a))


def test_lincomb_bit_exact(tiny):
    """Two-term and one-term constant combinations, rescaled and unrescaled, at two levels."""
    g, o, _ = tiny
    a, _ = _rand_ct(o, 16)
    b, _ = _rand_ct(o, 17, scale=2.0**40 * 0.997)
    for lvl in (a.level, 2):
        al, bl = o.lower(a, lvl), o.lower(b, lvl)
        ga, gb = g.import_(al.export(), al.scale), g.import_(bl.export(), bl.scale)
        for vb, T, rs in ((0.37, 2.0**40, True), (-2.5, 2.0**80 * 1.01, False)):
            _same(g, g.lincomb(ga, 1.25, gb, vb, T, rs), o.lincomb(al, 1.25, bl, vb, T, rs))
            _same(g, g.lincomb(ga, -0.75, None, 0.0, T, rs), o.lincomb(al, -0.75, None, 0.0, T, rs))


def test_products_and_rotations_bit_exact(tiny):
    g, o, steps = tiny
    a, _ = _rand_ct(o, 9)
    b, _ = _rand_ct(o, 10, level=5)
    ga, gb = g.import_(a.export(), a.scale), g.import_(b.export(), b.scale)
    _same(g, g.mul_relin(ga, gb), o.mul_relin(a, b))
    _same(g, g.mul_relin_rescale(ga, ga), o.mul_relin_rescale(a, a))
    # merged relinearise + rescale at a ragged level and at level 1 (result at level 0)
    _same(g, g.mul_relin_rescale(ga, gb), o.mul_relin_rescale(a, b))
    a1 = o.lower(a, 1)
    ga1 = g.import_(a1.export(), a1.scale)
    _same(g, g.mul_relin_rescale(ga1, ga1), o.mul_relin_rescale(a1, a1))
    for st in [1, 3, 5, steps[-1], o.slots - 4]:
        if st not in steps:
            continue
        _same(g, g.rotate(ga, st), o.rotate(a, st))
        _same(g, g.rotate(gb, st), o.rotate(b, st))


@pytest.mark.parametrize("level", [7, 4, 1, 0])
def test_key_switch_bit_exact(tiny, level):
    """Hybrid key switch at full and partial digit counts (ragged last digit)."""
    g, o, _ = tiny
    rng = np.random.default_rng(level)
    primes = [int(v) for v in o.primes]
    d = np.stack([rng.integers(0, primes[t], o.n, dtype=np.uint64) for t in range(level + 1)])
    gu = g.key_switch(0, d)
    ou = o.key_switch(0, d)
    assert np.array_equal(gu[0], ou[0]) and np.array_equal(gu[1], ou[1])


@pytest.mark.parametrize("name", ["p11", "p12", "p14", "p15"])
def test_other_sizes_key_switching_bit_exact(name):
    """N = 2^11 and 2^12 (the single-pass NTT of a whole limb per workgroup),
    2^14 (2^7 x 2^7) and 2^15 (2^7 x 2^8; their own shapes of the
    column-fused ModUp and ModDown and of the inner product's row pass): key
    switches at full and ragged digit counts, the merged relinearise +
    rescale, rotations and a whole Algorithm 1 match the oracle bit for bit."""
    g, o, steps = _pair(name, 2, 2)
    rng = np.random.default_rng(14)
    primes = [int(v) for v in o.primes]
    for level in (7, 4, 0):
        d = np.stack([rng.integers(0, primes[t], o.n, dtype=np.uint64) for t in range(level + 1)])
        gu, ou = g.key_switch(0, d), o.key_switch(0, d)
        assert np.array_equal(gu[0], ou[0]) and np.array_equal(gu[1], ou[1]), level
    a, _ = _rand_ct(o, 41)
    b, _ = _rand_ct(o, 42, level=5)
    ga, gb = g.import_(a.export(), a.scale), g.import_(b.export(), b.scale)
    _same(g, g.mul_relin_rescale(ga, gb), o.mul_relin_rescale(a, b))
    _same(g, g.mul_relin_rescale(ga, ga), o.mul_relin_rescale(a, a))
    for st in (1, 3):
        _same(g, g.rotate(gb, st), o.rotate(b, st))
    # 32 rotations in one launch: enough workgroups for the grouped base
    # conversions (a single key switch takes one output limb per workgroup);
    # uniform residues, since a key switch needs no encodable plaintext
    cs = []
    for i in range(32):
        lv = 7 - i % 3
        data = np.stack([np.stack([rng.integers(0, primes[t], o.n, dtype=np.uint64) for t in range(lv + 1)])
                         for _ in range(2)])
        cs.append(o.ct_import(data, 2.0**40))
    gs = g.rotate_batch([g.import_(c.export(), c.scale) for c in cs], [1 + 2 * (i % 2) for i in range(32)])
    for i, (gc, c) in enumerate(zip(gs, cs)):
        _same(g, gc, o.rotate(c, 1 + 2 * (i % 2)))
    print(f"[{name}] Algorithm 1, K = C = 2 (oracle and GPU)", flush=True)
    y, zo, zg = _argmax_pair(g, o, 2, 2, q=7)
    _same(g, zg, zo)


def test_refresh_bit_exact(tiny):
    g, o, _ = tiny
    a, _ = _rand_ct(o, 11, level=2)
    ga = g.import_(a.export(), a.scale)
    _same(g, g.refresh(ga, 1234, 3, owner=g.owner), o.refresh(a, 1234, 3))


def test_eval_odd9_bit_exact(tiny):
    g, o, _ = tiny
    f, gg = sign_coeffs()
    a, _ = _rand_ct(o, 12)
    ga = g.import_(a.export(), a.scale)
    _same(g, g.eval_odd9(ga, gg, 1.0, 2.0**40), o.eval_odd9(a, gg, 1.0, 2.0**40))
    _same(g, g.eval_odd9(ga, f, 0.5, 2.0**40 * 0.999), o.eval_odd9(a, f, 0.5, 2.0**40 * 0.999))


def _argmax_pair(g, o, K, C, cfg=9, q=0):
    y = W.logits(cfg, q, K, C)
    dmin, dmax = W.d_bounds(K)
    enc, ref = W.query_seeds(cfg, q)
    ct_o = o.encrypt_logits(y, enc)
    ct_g = g.encrypt(y, enc)
    zo = o.eval_argmax(ct_o, K, C, dmin, dmax, ref)
    zg = g.eval_argmax(ct_g, K, C, dmin, dmax, ref, owner=g.owner)
    return y, zo, zg


@pytest.mark.parametrize("K,C", [(1, 1), (1, 2), (2, 2), (3, 5), (4, 3), (8, 8)])
def test_argmax_bit_exact_tiny(tiny, K, C):
    """The whole Algorithm 1 (prompt sum, Eq. 5, duplication, QuickMax, Eq. 2) matches
    the oracle bit for bit, with padding (C, K not powers of two) and degenerate shapes."""
    g, o, _ = tiny
    y, zo, zg = _argmax_pair(g, o, K, C, q=K * 16 + C)
    _same(g, zg, zo)
    z, idx = g.decrypt(zg, C)
    zs = sim.t1_argmax(y, *W.d_bounds(K), o.slots)
    assert np.abs(z - zs).max() < 1e-3


@pytest.mark.parametrize("name", ["tiny_r6", "p13_r6"])
def test_argmax_refresh_below_top_bit_exact(name):
    """Refreshes re-encrypting at level 6 instead of the top (single-pass and two-pass
    NTT sizes): refresh and the whole Algorithm 1 match the oracle bit for bit."""
    g, o, _ = _pair(name, 4, 8)
    a, _ = _rand_ct(o, 31, level=2)
    ga = g.import_(a.export(), a.scale)
    r = o.refresh(a, 77, 2)
    assert r.level == 6
    _same(g, g.refresh(ga, 77, 2, owner=g.owner), r)
    y, zo, zg = _argmax_pair(g, o, 3, 5, q=5)
    _same(g, zg, zo)


def _packed_case(seed, shapes):
    blocks = [W.logits(9, seed * 100 + i, K, C) for i, (K, C) in enumerate(shapes)]
    lo = [W.d_bounds(K)[0] for K, _ in shapes]
    hi = [W.d_bounds(K)[1] for K, _ in shapes]
    return blocks, lo, hi


@pytest.mark.parametrize("name", ["tiny", "p13"])
def test_packed_argmax_bit_exact(name, tiny, p13):
    """Slot-packed Argmax (several queries in one ciphertext, Sec. 3.2): encryption and
    the whole evaluation match the oracle bit for bit; two packed ciphertexts in one
    batch give the same bits as each alone; every block decodes to its plaintext argmax."""
    g, o, _ = tiny if name == "tiny" else p13
    groups = [[(3, 5), (2, 3), (4, 2), (1, 4)], [(2, 2), (3, 3)]]
    if name == "p13":
        groups = [[(3, 4), (2, 3), (4, 2)], [(1, 2), (2, 4)]]
    cases = [_packed_case(20 + i, sh) for i, sh in enumerate(groups)]
    gcts, octs = [], []
    for i, (blocks, lo, hi) in enumerate(cases):
        octs.append(o.encrypt_packed(blocks, 50 + i))
        gcts.append(g.encrypt_packed(blocks, 50 + i))
        _same(g, gcts[-1], octs[-1])
    lo_all = [v for _, lo, _ in cases for v in lo]
    hi_all = [v for _, _, hi in cases for v in hi]
    outs = g.eval_argmax_packed(gcts, groups, lo_all, hi_all, [60, 61], owner=g.owner)
    for i, (blocks, lo, hi) in enumerate(cases):
        zo = o.eval_argmax_packed(octs[i], groups[i], lo, hi, 60 + i)
        _same(g, outs[i], zo)
        alone = g.eval_argmax_packed([gcts[i]], [groups[i]], lo, hi, [60 + i], owner=g.owner)[0]
        assert np.array_equal(g.export(alone), g.export(outs[i]))
        for (zb, idx), y, l, h in zip(g.decrypt_packed(outs[i], groups[i]), blocks, lo, hi):
            i0, _, margin = sim.t0_argmax(y)
            if margin / (h - l) >= 2.0**-10:
                assert idx == i0


@pytest.mark.parametrize("name", ["tiny43", "tiny52"])
def test_argmax_precise_sign_bit_exact(name):
    """Higher-precision Signs, (d_g, d_f) = (4, 3) and (5, 2) (seven polynomials per
    Sign): the whole Algorithm 1 matches the oracle bit for bit."""
    g, o, _ = _pair(name, 4, 8)
    for i, (K, C) in enumerate([(3, 5), (2, 2)]):
        y, zo, zg = _argmax_pair(g, o, K, C, q=400 + i)
        _same(g, zg, zo)


def test_argmax_large_n_bit_exact(tiny):
    """Large n: C = 200 classes (C' = 256, eight QuickMax steps, nine Signs) in the 512
    slots of N = 2^10: bit-exact with the oracle and the right index."""
    from paper_2502_00847_amd.secpe import Context
    p = _params("tiny")
    g, o = Context(p), Oracle.from_params(p)
    steps = g.argmax_steps(2, 256)
    g.keygen(SEED, steps)
    g.owner = g.key_owner()
    o.keygen(SEED, steps)
    y, zo, zg = _argmax_pair(g, o, 2, 200, q=500)
    _same(g, zg, zo)
    z, idx = g.decrypt(zg, 200)
    i0, _, margin = sim.t0_argmax(y)
    if margin / (W.d_bounds(2)[1] - W.d_bounds(2)[0]) >= 2.0**-10:
        assert idx == i0


@pytest.mark.parametrize("name,K,C", [("tiny", 2, 5), ("p13", 3, 4)])
def test_phoenix_bit_exact(name, K, C):
    """The comparison path (Phoenix: C Signs, C rotations) matches the oracle bit for
    bit at single-pass and two-pass NTT sizes, and decodes to the plaintext argmax."""
    from paper_2502_00847_amd.secpe import Context
    p = _params(name)
    g, o = Context(p), Oracle.from_params(p)
    steps = g.phoenix_steps(K, C)
    g.keygen(SEED, steps)
    g.owner = g.key_owner()
    o.keygen(SEED, steps)
    y = W.logits(9, 800 + C, K, C)
    lo, hi = W.d_bounds(K)
    enc, ref = W.query_seeds(9, 800 + C)
    zg = g.eval_argmax_phoenix(g.encrypt(y, enc), K, C, lo, hi, ref, owner=g.owner)
    zo = o.eval_argmax_phoenix(o.encrypt_logits(y, enc), K, C, lo, hi, ref)
    _same(g, zg, zo)
    cnt = g.counters()
    assert cnt["sign"] == C and cnt["rotate"] == (K - 1).bit_length() + C
    z, idx = g.decrypt(zg, C)
    i0, _, margin = sim.t0_argmax(y)
    if margin / (hi - lo) >= 2.0**-8:
        assert idx == i0


def test_argmax_toy_config(p13):
    """Toy-shaped parameters with the two-pass NTT: K=4, C=2 (config 1 shape)."""
    g, o, _ = p13
    y, zo, zg = _argmax_pair(g, o, 4, 2, cfg=1, q=0)
    _same(g, zg, zo)
    z, idx = g.decrypt(zg, 2)
    assert idx == sim.t0_argmax(y)[0]


def test_batch_equals_one_at_a_time(tiny):
    """Uneven (K, C) in one batched evaluation give the same bits as alone."""
    g, o, _ = tiny
    shapes = [(3, 5), (8, 2), (1, 7), (4, 4), (2, 3)]
    cts, Ks, Cs, dmin, dmax, seeds = [], [], [], [], [], []
    for i, (K, C) in enumerate(shapes):
        y = W.logits(11, i, K, C)
        enc, ref = W.query_seeds(11, i)
        cts.append(g.encrypt(y, enc))
        Ks.append(K)
        Cs.append(C)
        lo, hi = W.d_bounds(K)
        dmin.append(lo)
        dmax.append(hi)
        seeds.append(ref)
    outs = g.eval_argmax_batch(cts, Ks, Cs, dmin, dmax, seeds, owner=g.owner)
    for i in range(len(shapes)):
        alone = g.eval_argmax(cts[i], Ks[i], Cs[i], dmin[i], dmax[i], seeds[i], owner=g.owner)
        assert outs[i].level == alone.level and outs[i].scale == alone.scale
        assert np.array_equal(g.export(outs[i]), g.export(alone))


def test_autotune_keeps_bits(p13):
    """Every autotuner candidate schedule gives the same ciphertexts (two-pass NTT size)."""
    g, o, _ = p13
    shapes = [(4, 4), (3, 2), (2, 3)]
    qs = [(K, C, W.logits(9, 300 + i, K, C), W.query_seeds(9, 300 + i)) for i, (K, C) in enumerate(shapes)]
    cts = [g.encrypt(y, enc) for K, C, y, (enc, _) in qs]
    args = ([K for K, *_ in qs], [C for _, C, *_ in qs], [W.d_bounds(K)[0] for K, *_ in qs],
            [W.d_bounds(K)[1] for K, *_ in qs], [ref for *_, (_, ref) in qs])
    ws = g.workspace(args[0], args[1])
    before = [g.export(z) for z in g.eval_argmax_batch(cts, *args, ws=ws, owner=g.owner)]
    outs = [g.new_ct() for _ in cts]
    chosen, cands = g.autotune(cts, *args, ws=ws, outs=outs, owner=g.owner)
    assert chosen in [c["index"] for c in cands] and all(c["ms"] > 0 for c in cands)
    assert len(cands) == 7   # the default and each of the six knobs flipped in turn
    assert all(np.array_equal(g.export(a), b) for a, b in zip(outs, before))
    after = [g.export(z) for z in g.eval_argmax_batch(cts, *args, ws=ws, owner=g.owner)]
    assert all(np.array_equal(a, b) for a, b in zip(after, before))


def test_graph_replay_is_deterministic(tiny):
    g, o, _ = tiny
    shapes = [(3, 5), (8, 2), (2, 3)]
    cts, Ks, Cs, dmin, dmax, seeds = [], [], [], [], [], []
    for i, (K, C) in enumerate(shapes):
        y = W.logits(12, i, K, C)
        enc, ref = W.query_seeds(12, i)
        cts.append(g.encrypt(y, enc))
        Ks.append(K)
        Cs.append(C)
        lo, hi = W.d_bounds(K)
        dmin.append(lo)
        dmax.append(hi)
        seeds.append(ref)
    ws = g.workspace(Ks, Cs)
    outs = [g.new_ct() for _ in shapes]
    eager = [g.export(c) for c in g.eval_argmax_batch(cts, Ks, Cs, dmin, dmax, seeds, ws=ws, outs=outs, owner=g.owner)]
    for rep in range(3):
        got = g.eval_argmax_batch(cts, Ks, Cs, dmin, dmax, seeds, ws=ws, outs=outs, graph=True, owner=g.owner)
        g.sync()
        for e, c in zip(eager, got):
            assert np.array_equal(g.export(c), e)
        # eager work between replays
        g.eval_argmax(cts[0], Ks[0], Cs[0], dmin[0], dmax[0], seeds[0], owner=g.owner)


def test_without_key_owner_the_evaluation_stops_at_a_refresh(tiny):
    """Sec. 3.1: the server holds no secret.  An evaluation that needs a
    refresh and has no key owner (and no bootstrapping) stops with
    SECPE_ENOLEVEL before queuing work; the server refuses such a request at
    submission; with the owner the same call runs."""
    from paper_2502_00847_amd.secpe import SecpeError, Server
    g, o, _ = tiny
    K, C = 4, 3
    y = W.logits(1, 0, K, C)
    lo, hi = W.d_bounds(K)
    ct = g.encrypt(y, 5)
    with pytest.raises(SecpeError, match="error -3"):
        g.eval_argmax(ct, K, C, lo, hi, 6)
    with pytest.raises(SecpeError, match="error -3"):
        g.eval_argmax_batch([ct, ct], [K, K], [C, C], [lo, lo], [hi, hi], [6, 7])
    with pytest.raises(SecpeError, match="error -3"):
        g.refresh(ct, 1, 0, owner=None)
    srv = Server(g, 4 * g.workspace_bytes([K], [C]), max_active=4)
    with pytest.raises(SecpeError, match="error -3"):
        srv.submit(ct, K, C, lo, hi, 6)
    z = g.eval_argmax(ct, K, C, lo, hi, 6, owner=g.owner)
    assert g.counters()["refresh"] >= 1
    assert g.decrypt(z, C)[1] == sim.t0_argmax(y)[0]


def test_graph_is_recaptured_after_new_keys():
    """A captured graph bakes in the key pointers: new keys (keygen) or another
    key owner discard it, so a replay after them equals an eager evaluation
    with the new keys."""
    from paper_2502_00847_amd.secpe import Context
    g = Context(_params("tiny"))
    g.keygen(SEED, g.argmax_steps(4, 4))
    owner = g.key_owner()
    shapes = [(3, 3), (2, 4)]
    ys = [W.logits(14, i, K, C) for i, (K, C) in enumerate(shapes)]
    Ks, Cs = [K for K, _ in shapes], [C for _, C in shapes]
    lo, hi = [W.d_bounds(K)[0] for K in Ks], [W.d_bounds(K)[1] for K in Ks]
    ws = g.workspace(Ks, Cs)
    outs = [g.new_ct() for _ in shapes]
    cts = [g.encrypt(y, 40 + i) for i, y in enumerate(ys)]
    first = [g.export(c) for c in g.eval_argmax_batch(cts, Ks, Cs, lo, hi, [50, 51], ws=ws, outs=outs, graph=True,
                                                       owner=owner)]
    g.sync()
    old_sk = g.sk
    g.keygen(SEED + 1, g.argmax_steps(4, 4))      # new secret and switching keys
    owner2 = g.key_owner()
    # the same input buffers now hold encryptions under the new secret
    import torch
    for i, y in enumerate(ys):
        new = g.encrypt(y, 40 + i)
        g.sync()                                  # encryption is asynchronous on the context's stream
        cts[i].buf.copy_(new.buf)
    torch.cuda.synchronize()
    eager = [g.export(c) for c in g.eval_argmax_batch(cts, Ks, Cs, lo, hi, [50, 51], ws=ws, outs=outs,
                                                       owner=owner2)]
    for rep in range(2):
        got = g.eval_argmax_batch(cts, Ks, Cs, lo, hi, [50, 51], ws=ws, outs=outs, graph=True, owner=owner2)
        g.sync()
        for e, c in zip(eager, got):
            assert np.array_equal(g.export(c), e)
    assert not all(np.array_equal(a, b) for a, b in zip(first, eager))
    for (K, C), y, c in zip(shapes, ys, got):
        assert g.decrypt(c, C)[1] == sim.t0_argmax(y)[0]
    del old_sk


def test_keyswitch_traffic_counts_each_key_once_per_launch(tiny):
    """The algorithmic key-switch bytes of a launch: (l+1) limbs read and
    2 (l+1) written per key switch, each distinct key's 2 dnum (l+1+alpha)
    limbs once, however many key switches of the launch share it."""
    g, o, _ = tiny
    cts = [g.encrypt(np.zeros((2, 2)), 100 + i) for i in range(4)]
    nc, alpha = g.n_q, g.n_p
    nd = -(-nc // alpha)
    limb = g.N * 8
    key = 2 * nd * (nc + alpha)
    g.rotate_batch(cts, [3, 3, 3, 3])
    assert g.keyswitch_traffic() == (4 * 3 * nc + key) * limb
    g.rotate_batch(cts, [3, 5, 3, 5])
    assert g.keyswitch_traffic() == (4 * 3 * nc + 2 * key) * limb
    g.sync()


def test_segment_profile_alternates_computation_and_refresh(tiny):
    """The segment profiler times an evaluation between refreshes: one
    interval before the first refresh, then each refresh and the computation
    after it."""
    g, o, _ = tiny
    K, C = 4, 3
    y = W.logits(1, 3, K, C)
    lo, hi = W.d_bounds(K)
    ct = g.encrypt(y, 8)
    g.profile_begin("segments")
    g.eval_argmax(ct, K, C, lo, hi, 9, owner=g.owner)
    prof = g.profile_end()
    seg = g.profile_segments()
    n_ref = g.counters()["refresh"]
    assert n_ref >= 1 and len(seg) == 2 * n_ref + 1
    assert all(t >= 0 for t in seg) and abs(sum(seg) - prof["ms"]) < 1e-6 * max(1.0, prof["ms"])


def test_errors_are_reported(tiny):
    from paper_2502_00847_amd.secpe import SecpeError
    g, o, _ = tiny
    ct = g.encrypt(np.zeros((2, 2)), 1)
    with pytest.raises(SecpeError):
        g.rotate(ct, 1000)          # no key for this rotation
    with pytest.raises(SecpeError):
        g.eval_argmax(ct, 64, 64, -1, 1, 0, owner=g.owner)   # K' C' exceeds the slots
    with pytest.raises(SecpeError):
        g.eval_argmax(ct, 2, 2, 1.0, 1.0, 0, owner=g.owner)  # empty normalisation range
    # slot-packed mode: too many blocks for the slots, bad shapes, bad bounds
    with pytest.raises(SecpeError):
        g.encrypt_packed([np.zeros((4, 8))] * 17, 1)          # 17 blocks of 32 > 512 slots
    with pytest.raises(SecpeError):
        g.packed_shape([(0, 2)])
    packed = g.encrypt_packed([np.zeros((2, 2))] * 2, 1)
    with pytest.raises(SecpeError):
        g.eval_argmax_packed([packed], [[(2, 2)] * 200], [-1.0] * 200, [1.0] * 200, [0], owner=g.owner)
    with pytest.raises(SecpeError):
        g.eval_argmax_packed([packed], [[(2, 2), (2, 2)]], [-1.0, 1.0], [1.0, 1.0], [0], owner=g.owner)
