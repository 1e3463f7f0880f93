"""GPU parity at the full sizes of the workloads (N = 2^16, 24 chain primes,
8 special primes, dnum 3) and at the toy configuration.

* single operations at the top level and at a ragged level are bit-exact with
  the oracle run here on the same inputs;
* whole encrypted Argmax evaluations are compared with digests the oracle
  wrote (tests/golden/argmax_digests.json, made by tests/golden/make_golden.py,
  which calls only oracle/);
* the batched launch gives the same bits as one query at a time, and every
  decrypted index of a 256-query batch is checked against the plaintext argmax.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import workload as W
from oracle import sim
from oracle.ckks import Oracle, sign_coeffs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "argmax_digests.json")


def _digest(arr):
    return hashlib.sha256(np.ascontiguousarray(arr).astype("<u8").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def full_gpu():
    from paper_2502_00847_amd.secpe import Context
    g = Context(W.PARAMS["full"])
    g.keygen(W.KEYGEN_SEED, g.argmax_steps(16, 14))
    g.owner = g.key_owner()
    return g


@pytest.fixture(scope="module")
def full_pair():
    """GPU and oracle contexts at full size with the relinearisation key and two rotation keys."""
    from paper_2502_00847_amd.secpe import Context
    p = W.PARAMS["full"]
    g = Context(p)
    o = Oracle.from_params(p)
    steps = [1, 4096]
    print("[full_pair] oracle keygen", flush=True)
    g.keygen(7, steps)
    g.owner = g.key_owner()
    o.keygen(7, steps)
    return g, o


def _same(g, gct, oct_):
    assert (gct.level, gct.scale) == (oct_.level, oct_.scale)
    assert np.array_equal(g.export(gct), oct_.export())


def test_full_keys_and_encrypt(full_pair):
    g, o = full_pair
    assert np.array_equal(g.secret(), o.secret())
    for t in (0, 23, 31):
        assert np.array_equal(g.key_limb(0, 2, 0, t), o.key_limb(0, 2, 0, t))
    d = W.query(2, 0)
    _same(g, g.encrypt(d["logits"], d["encrypt_seed"]), o.encrypt_logits(d["logits"], d["encrypt_seed"]))


def test_full_rotate_and_product_top_level(full_pair):
    g, o = full_pair
    z = np.random.default_rng(1).uniform(-1, 1, o.slots)
    ct = o.encrypt(o.encode(z[:256], 2.0**50), 2.0**50, 5)
    gct = g.import_(ct.export(), ct.scale)
    _same(g, g.rotate(gct, 4096), o.rotate(ct, 4096))
    _same(g, g.mul_relin_rescale(gct, gct), o.mul_relin_rescale(ct, ct))


@pytest.mark.parametrize("level", [23, 12, 1])
def test_full_key_switch_levels(full_pair, level):
    """Three full digits at level 23; 8+5 primes at level 12 (ragged); one digit of 2 at level 1."""
    g, o = full_pair
    rng = np.random.default_rng(level)
    pr = [int(v) for v in o.primes]
    d = np.stack([rng.integers(0, pr[t], o.n, dtype=np.uint64) for t in range(level + 1)])
    gu, ou = g.key_switch(0, d), o.key_switch(0, d)
    assert np.array_equal(gu[0], ou[0]) and np.array_equal(gu[1], ou[1])


def test_full_batched_ntt_and_rotations(full_pair):
    """The kernel microbenchmark's entry points: batched inverse NTT of whole
    ciphertexts equals the oracle's coefficient-domain residues, forward NTT
    restores them; batched rotations with different keys equal the oracle's."""
    g, o = full_pair
    cts, gcts = [], []
    for i, lvl in enumerate((23, 23, 11)):
        z = np.random.default_rng(40 + i).uniform(-1, 1, 128)
        c = o.lower(o.encrypt(o.encode(z, 2.0**50), 2.0**50, 40 + i), lvl)
        cts.append(c)
        gcts.append(g.import_(c.export(), c.scale))
    g.ntt_cts(gcts, inverse=True)
    g.sync()
    for c, gc in zip(cts, gcts):
        raw = gc.buf.view(2, g.n_q, g.N)[:, : c.level + 1].cpu().numpy().astype(np.uint64)
        assert np.array_equal(raw, c.export())
    g.ntt_cts(gcts, inverse=False)
    for c, gc in zip(cts, gcts):
        assert np.array_equal(g.export(gc), c.export())
    steps = [1, 4096, 1]
    outs = g.rotate_batch(gcts, steps)
    for c, st, out in zip(cts, steps, outs):
        _same(g, out, o.rotate(c, st))


def test_full_refresh_and_poly(full_pair):
    g, o = full_pair
    f, gg = sign_coeffs()
    z = np.random.default_rng(2).uniform(-1, 1, 64)
    ct = o.encrypt(o.encode(z, 2.0**50), 2.0**50, 6)
    low = o.lower(ct, 3)
    gl = g.import_(low.export(), low.scale)
    _same(g, g.refresh(gl, 99, 1, owner=g.owner), o.refresh(low, 99, 1))


@pytest.mark.parametrize("level", [23, 12, 1])
def test_full_lincomb_levels(full_pair, level):
    """Constant combinations on the two-pass transform sizes: a rescaled one is
    formed in the rescale's row-pass epilogue, an unrescaled one elementwise;
    one and two terms, at the top, a middle and the lowest rescalable level."""
    g, o = full_pair
    rng = np.random.default_rng(60 + level)
    sb = 2.0**50 * 0.997
    a = o.lower(o.encrypt(o.encode(rng.uniform(-1, 1, 64), 2.0**50), 2.0**50, 61), level)
    b = o.lower(o.encrypt(o.encode(rng.uniform(-1, 1, 64), sb), sb, 62), level)
    ga, gb = g.import_(a.export(), a.scale), g.import_(b.export(), b.scale)
    for T, rs in ((2.0**50, True), (2.0**100 * 1.01, False)):
        _same(g, g.lincomb(ga, 1.25, gb, 0.37, T, rs), o.lincomb(a, 1.25, b, 0.37, T, rs))
        _same(g, g.lincomb(ga, -0.75, None, 0.0, T, rs), o.lincomb(a, -0.75, None, 0.0, T, rs))


def test_full_eval_odd9(full_pair):
    """One Sign polynomial on the two-pass sizes (fused squares, the degree-2
    sum that forms its addend combination, combinations rescaled in the
    epilogue, merged relinearise + rescale), for g and for f with the Max gain."""
    g, o = full_pair
    f, gg = sign_coeffs()
    z = np.random.default_rng(63).uniform(-1, 1, 64)
    a = o.lower(o.encrypt(o.encode(z, 2.0**50), 2.0**50, 64), 8)
    ga = g.import_(a.export(), a.scale)
    _same(g, g.eval_odd9(ga, gg, 1.0, 2.0**50), o.eval_odd9(a, gg, 1.0, 2.0**50))
    _same(g, g.eval_odd9(ga, f, 0.5, 2.0**50 * 0.999), o.eval_odd9(a, f, 0.5, 2.0**50 * 0.999))


@pytest.mark.parametrize("case", ["config2_full", "config3_full_q0"])
def test_full_argmax_matches_oracle_digest(full_gpu, golden, case):
    """Config 2 (K=8, C=4, N=2^16, dnum 3): the whole encrypted Argmax is bit-exact with the oracle."""
    rec = golden[case]
    g = full_gpu
    d = W.query(rec["config"], rec["query"])
    ct = g.encrypt(d["logits"], d["encrypt_seed"])
    assert _digest(g.export(ct)) == rec["input_sha256"]
    z = g.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"], owner=g.owner)
    assert (z.level, z.scale) == (rec["level"], rec["scale"])
    assert _digest(g.export(z)) == rec["output_sha256"]
    zz, idx = g.decrypt(z, d["C"])
    assert np.allclose(zz, rec["z"], rtol=0, atol=1e-9)
    assert idx == sim.t0_argmax(d["logits"])[0]
    cnt = g.counters()
    for k in ("sign", "rotate", "relin", "refresh", "max"):
        assert cnt[k] == rec["counters"][k], k


def _batch_digests(g, recs):
    """Evaluate the golden cases in one batched launch; check each against the oracle's digest."""
    ds = [W.query(r["config"], r["query"]) for r in recs]
    cts = [g.encrypt(d["logits"], d["encrypt_seed"]) for d in ds]
    for ct, r in zip(cts, recs):
        assert _digest(g.export(ct)) == r["input_sha256"]
    outs = g.eval_argmax_batch(cts, [d["K"] for d in ds], [d["C"] for d in ds], [d["d_min"] for d in ds],
                               [d["d_max"] for d in ds], [d["refresh_seed"] for d in ds], owner=g.owner)
    bad = []
    for r, d, z in zip(recs, ds, outs):
        ok = (z.level, z.scale) == (r["level"], r["scale"]) and _digest(g.export(z)) == r["output_sha256"]
        zz, idx = g.decrypt(z, d["C"])
        ok = ok and np.allclose(zz, r["z"], rtol=0, atol=1e-9)
        i0, _, margin = sim.t0_argmax(d["logits"])
        if margin / (d["d_max"] - d["d_min"]) >= 2.0**-10:
            ok = ok and idx == i0
        if not ok:
            bad.append((r["config"], r["query"], d["K"], d["C"]))
    assert not bad, bad


def test_config3_sample_matches_oracle_digests_batched(full_gpu, golden):
    """24 queries of the 256-query batch, two of every padded shape (K', C') in
    {4, 8, 16} x {2, 4, 8, 16} (refreshes at level 14 for C' = 8, 16 included),
    evaluated in one batched launch: every output ciphertext is bit-exact with
    the oracle's."""
    recs = [r for k, r in sorted(golden.items()) if k.startswith("config3_full_q")]
    assert len(recs) >= 16
    shapes = {(1 << (r["K"] - 1).bit_length(), 1 << (r["C"] - 1).bit_length()) for r in recs}
    assert len(shapes) == 12
    _batch_digests(full_gpu, recs)


def test_config5_full_matches_oracle_digests():
    """Serving-mix shapes at N = 2^16 with K' or C' = 32 (five prompt-sum
    doublings, five QuickMax steps): bit-exact with the oracle's digests."""
    from paper_2502_00847_amd.secpe import Context
    with open(GOLDEN) as f:
        recs = [r for k, r in sorted(json.load(f).items()) if k.startswith("config5_full_q")]
    assert len(recs) == 3
    g = Context(W.PARAMS["full"])
    g.keygen(W.KEYGEN_SEED, g.argmax_steps(32, 20))
    g.owner = g.key_owner()
    _batch_digests(g, recs)


def test_every_schedule_keeps_the_config2_bits(full_gpu, golden):
    """Each knob of the autotuner on its own (two-tile column passes, forward
    and inverse; two output limbs per ModUp or ModDown workgroup; NTT job
    groups) gives the oracle's config-2 ciphertext at N = 2^16."""
    rec = golden["config2_full"]
    g = full_gpu
    d = W.query(2, 0)
    ct = g.encrypt(d["logits"], d["encrypt_seed"])
    try:
        for cand in (1, 2, 4, 8, 16, 32, 28, 63):
            g.set_schedule(cand)
            z = g.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"], owner=g.owner)
            assert _digest(g.export(z)) == rec["output_sha256"], cand
    finally:
        g.set_schedule(0)


def test_toy_argmax_matches_oracle_digest(golden):
    """Config 1: N=2^13, 8 x 30-bit primes + 1 special prime, scale 2^30, K=4, C=2."""
    from paper_2502_00847_amd.secpe import Context
    rec = golden["config1_toy"]
    g = Context(W.PARAMS["toy"])
    g.keygen(W.KEYGEN_SEED, g.argmax_steps(4, 2))
    g.owner = g.key_owner()
    d = W.query(1, 0)
    ct = g.encrypt(d["logits"], d["encrypt_seed"])
    z = g.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"], owner=g.owner)
    assert _digest(g.export(z)) == rec["output_sha256"]
    zz, idx = g.decrypt(z, 2)
    assert idx == sim.t0_argmax(d["logits"])[0]


def test_toy_deep_argmax_without_refresh(golden):
    """Config 1 on a 36-prime chain (alpha = 4, dnum = 9): the whole of Algorithm 1
    non-interactively, no refresh, bit-identical to the oracle."""
    from paper_2502_00847_amd.secpe import Context
    rec = golden["config1_toy_deep"]
    g = Context(W.PARAMS["toy_deep"])
    g.keygen(W.KEYGEN_SEED, g.argmax_steps(4, 2))
    d = W.query(1, 0)
    ct = g.encrypt(d["logits"], d["encrypt_seed"])
    # no key owner: the evaluation is the server's alone
    z = g.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"])
    assert z.level == rec["level"] and z.scale == rec["scale"]
    assert _digest(g.export(z)) == rec["output_sha256"]
    cnt = g.counters()
    assert cnt["refresh"] == 0 == rec["counters"]["refresh"]
    for k in ("sign", "rotate", "relin", "key_switch", "max"):
        assert cnt[k] == rec["counters"][k], k
    zz, idx = g.decrypt(z, 2)
    assert idx == sim.t0_argmax(d["logits"])[0]


def test_config3_batch_indices_and_bit_identity(full_gpu):
    """256 queries with uneven (K, C) in batched launches: every decrypted index
    equals the plaintext argmax when the normalised top-2 margin is at least
    2^-10 (the Sign's stated index precision); sampled queries give the same
    bits alone as in the batch."""
    g = full_gpu
    qs = [W.query(3, i) for i in range(256)]
    cts = [g.encrypt(q["logits"], q["encrypt_seed"]) for q in qs]
    outs = []
    for s in range(0, 256, 64):
        grp = list(range(s, s + 64))
        outs += g.eval_argmax_batch([cts[i] for i in grp], [qs[i]["K"] for i in grp], [qs[i]["C"] for i in grp],
                                    [qs[i]["d_min"] for i in grp], [qs[i]["d_max"] for i in grp],
                                    [qs[i]["refresh_seed"] for i in grp], owner=g.owner)
    bad = []
    for i, (q, o) in enumerate(zip(qs, outs)):
        z, idx = g.decrypt(o, q["C"])
        i0, _, margin = sim.t0_argmax(q["logits"])
        if margin / (q["d_max"] - q["d_min"]) >= 2.0**-10 and idx != i0:
            bad.append(i)
    assert not bad, bad
    for i in (0, 37, 130, 255):
        alone = g.eval_argmax(cts[i], qs[i]["K"], qs[i]["C"], qs[i]["d_min"], qs[i]["d_max"], qs[i]["refresh_seed"], owner=g.owner)
        assert np.array_equal(g.export(alone), g.export(outs[i]))


def test_config3_packed_indices(full_gpu):
    """The 256 config-3 queries packed 128 per ciphertext (blocks of 256 slots, K' = C' = 16):
    every block's decrypted index equals the plaintext argmax at normalised margin >= 2^-10."""
    g = full_gpu
    qs = [W.query(3, i) for i in range(256)]
    shapes = [(q["K"], q["C"]) for q in qs]
    per, kp, cp, bsz = g.packed_shape(shapes)
    assert per == 128 and (kp, cp, bsz) == (16, 16, 256)
    groups = [shapes[i:i + per] for i in range(0, 256, per)]
    cts = [g.encrypt_packed([q["logits"] for q in qs[i:i + per]], 7000 + i) for i in range(0, 256, per)]
    outs = g.eval_argmax_packed(cts, groups, [q["d_min"] for q in qs], [q["d_max"] for q in qs], [8000, 8001], owner=g.owner)
    bad = []
    for j, (ct, grp) in enumerate(zip(outs, groups)):
        for b, (zb, idx) in enumerate(g.decrypt_packed(ct, grp)):
            q = qs[j * per + b]
            i0, _, margin = sim.t0_argmax(q["logits"])
            if margin / (q["d_max"] - q["d_min"]) >= 2.0**-10 and idx != i0:
                bad.append(j * per + b)
    assert not bad, bad
