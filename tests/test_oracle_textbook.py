"""The oracle's merged relinearise-and-rescale against the textbook evaluator.

The oracle (and the HIP path it pins bit for bit) relinearises and rescales a
product in one division by P q_l, and relinearises each Sign polynomial's
last sum x^4 B + x^8 C + A once, with A and Max's (a+b)/2 added before that
division (five key switches per polynomial).  The textbook evaluator of
Sec. 2.2 does tensor, relinearise, rescale for every product (six).  Both run
Algorithm 1 (Sec. 3.2) on the same seeded inputs here, on config 1, on a
C' = 8 shape and on config 2.  The bound on how far they may differ comes
from oracle/noise.py: every rounding step's residues give the message a
noise of known variance (N/2)(1 + h) V / Delta^2 per slot, pushed through
Algorithm 1 in FP64 by Monte Carlo; the check is 6 standard deviations per
slot.  The same model bounds each evaluator's distance from the noiseless
FP64 run (T1), so a wrong term in either evaluator, or a model that
understates the noise, fails here.
"""
import json
import os

import numpy as np
import pytest

import workload as W
from oracle import noise, sim
from oracle.ckks import Oracle, argmax_rotation_steps

K_SIGMA = 6.0


def _run(params, q, textbook):
    o = Oracle.from_params(params)
    o.set_textbook(textbook)
    o.keygen(W.KEYGEN_SEED, argmax_rotation_steps(q["K"], q["C"], o.slots))
    h = int(np.count_nonzero(o.secret()))
    z = o.eval_argmax(o.encrypt_logits(q["logits"], q["encrypt_seed"]), q["K"], q["C"], q["d_min"], q["d_max"],
                      q["refresh_seed"])
    return o.decrypt_decode(z, q["C"]), (z.level, z.scale), o.counters(), h


def _query(cfg, i, K=None, C=None):
    if K is None:
        return W.query(cfg, i)
    y = W.logits(cfg, i, K, C)
    enc, ref = W.query_seeds(cfg, i)
    lo, hi = W.d_bounds(K)
    return dict(K=K, C=C, logits=y, encrypt_seed=enc, refresh_seed=ref, d_min=lo, d_max=hi)


def _check(params, q, seed):
    zm, lsm, cm, h = _run(params, q, 0)
    zt, lst, ct, h2 = _run(params, q, 1)
    assert h == h2
    # same data flow: levels, scales, Signs, polynomials, rotations, refreshes
    assert lsm == lst
    for k in ("sign", "rotate", "refresh", "poly", "max"):
        assert cm[k] == ct[k], k
    # six key switches per polynomial against five, one per Max product in both
    assert ct["relin"] == cm["relin"] + cm["poly"]
    assert cm["relin"] == 5 * cm["poly"] + cm["max"]
    s = noise.argmax_noise_samples(q["logits"], q["d_min"], q["d_max"], params, h, n_pairs=200, seed=seed)
    t1 = sim.t1_argmax(q["logits"], q["d_min"], q["d_max"], (1 << params["log_n"]) // 2)[:q["C"]]
    assert np.abs(noise.noiseless(q["logits"], q["d_min"], q["d_max"], params) - t1).max() < 1e-12
    bound = K_SIGMA * (s["merged"] - s["textbook"]).std(axis=0)
    assert np.all(np.abs(zm - zt) <= bound), (np.abs(zm - zt), bound)
    for z, mode in ((zm, "merged"), (zt, "textbook")):
        dev = s[mode] - t1
        lim = np.abs(dev.mean(axis=0)) + K_SIGMA * dev.std(axis=0)
        assert np.all(np.abs(z - t1) <= lim), (mode, np.abs(z - t1), lim)
    i0 = sim.t0_argmax(q["logits"])[0]
    assert int(np.argmax(zm)) == int(np.argmax(zt)) == i0
    return np.abs(zm - zt).max(), bound.max()


@pytest.mark.parametrize("i", [0, 1])
def test_textbook_matches_merged_config1(i):
    _check(dict(W.PARAMS["toy"]), _query(1, i), seed=i)


@pytest.mark.parametrize("i", [0, 1, 2])
def test_textbook_matches_merged_c8(i):
    """C = 7 classes (C' = 8, three Max steps) on the N = 2^10 set."""
    _check(dict(W.PARAMS["tiny"]), _query(7, i, K=3, C=7), seed=100 + i)


@pytest.mark.slow
@pytest.mark.skipif(not os.environ.get("SECPE_SLOW_ORACLE"), reason="about 7 minutes of CPU; set SECPE_SLOW_ORACLE=1")
def test_textbook_matches_merged_config2_live():
    """Config 2: N = 2^16, 24 + 8 primes, K = 8, C = 4 (three minutes per evaluator)."""
    _check(dict(W.PARAMS["full"]), W.query(2, 0), seed=200)


def test_textbook_matches_merged_config2_stored():
    """Config 2 from the oracle's stored results of both evaluators
    (tests/golden/make_golden.py): z within the derived bound of each other
    and of T1, the same level, scale and index, six key switches per
    polynomial against five."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "argmax_digests.json")))
    m, t = gold["config2_full"], gold["config2_full_textbook"]
    params = dict(W.PARAMS["full"])
    q = W.query(2, 0)
    assert (m["level"], m["scale"]) == (t["level"], t["scale"])
    cm, ct = m["counters"], t["counters"]
    for k in ("sign", "rotate", "refresh", "poly", "max"):
        assert cm[k] == ct[k], k
    assert ct["relin"] == cm["relin"] + cm["poly"]
    zm, zt = np.array(m["z"]), np.array(t["z"])
    s = noise.argmax_noise_samples(q["logits"], q["d_min"], q["d_max"], params, m["secret_weight"], n_pairs=200,
                                   seed=200)
    t1 = sim.t1_argmax(q["logits"], q["d_min"], q["d_max"], (1 << params["log_n"]) // 2)[:q["C"]]
    assert np.all(np.abs(zm - zt) <= K_SIGMA * (s["merged"] - s["textbook"]).std(axis=0))
    for z, mode in ((zm, "merged"), (zt, "textbook")):
        dev = s[mode] - t1
        assert np.all(np.abs(z - t1) <= np.abs(dev.mean(axis=0)) + K_SIGMA * dev.std(axis=0)), mode
    i0 = sim.t0_argmax(q["logits"])[0]
    assert int(np.argmax(zm)) == int(np.argmax(zt)) == i0


def test_noise_model_detects_a_wrong_term():
    """A plausible slip in an evaluator (a Sign polynomial's c_3 term scaled by
    1 + 2^-10) moves z by far more than the bound: the check has teeth."""
    params = dict(W.PARAMS["tiny"])
    q = _query(7, 0, K=3, C=7)
    s = noise.argmax_noise_samples(q["logits"], q["d_min"], q["d_max"], params, 682, n_pairs=200, seed=5)
    bound = K_SIGMA * (s["merged"] - s["textbook"]).std(axis=0)
    f_bad = np.array(sim.F4)
    f_bad[1] *= 1.0 + 2.0**-10
    z_ok = sim.t1_argmax(q["logits"], q["d_min"], q["d_max"], 512)[:7]
    orig = sim.F4.copy()
    try:
        sim.F4[:] = f_bad
        z_bad = sim.t1_argmax(q["logits"], q["d_min"], q["d_max"], 512)[:7]
    finally:
        sim.F4[:] = orig
    assert np.any(np.abs(z_bad - z_ok) > bound)
