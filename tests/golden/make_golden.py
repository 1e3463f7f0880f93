"""Write tests/golden/argmax_digests.json from the CPU oracle only.

For each case the oracle encrypts the seeded logits, evaluates the encrypted
Argmax (Algorithm 1) and records: the SHA-256 of the output ciphertext in the
coefficient domain (canonical residues, uint64 little-endian, [2][level+1][N]),
its level and scale, the decrypted z and the operation counts.  The GPU parity
test recomputes the same digest from the HIP path.

Cases:
  config 1   toy N=2^13, 8 x 30-bit primes, K=4, C=2; and on 36 primes
             (alpha = 4) with no refresh at all;
  config 2   N=2^16, 24 x 50-bit primes, dnum 3, K=8, C=4, margin >= 0.05,
             with the default evaluator and with the textbook one (every
             product relinearised, then rescaled);
  config 3   24 queries of the 256-query batch (N=2^16): the first two of
             every padded shape (K', C') in {4, 8, 16} x {2, 4, 8, 16};
  config 5   three requests of the serving mix at N=2^16 with K' or C' = 32;
  boot13     bootstrapping at N=2^13 (the p13_boot set): one bootstrap of a
             seeded level-3 ciphertext, the sparse-slot bootstrap (n = 32) of
             the same ciphertext, and Algorithm 1 (K=2, C=2) with every
             refresh a (sparse-slot) bootstrap (the oracle takes about ten
             minutes per full bootstrap here); and the window-packed
             bootstrap of three seeded ciphertexts at levels 3, 2, 3.
Each case keys its own oracle with the rotations its shape needs (a key
depends only on the seed and its Galois element, so these equal the keys of
any larger set).  Cases run in parallel processes.
Run from the repository root: python tests/golden/make_golden.py [names...]
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workload as W  # noqa: E402
from oracle.ckks import Oracle, argmax_rotation_steps  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "argmax_digests.json")


def _pow2(v):
    return 1 << max(0, (v - 1).bit_length())


def config3_sample(per_shape=2):
    """The first per_shape queries of every padded shape in the 256-query batch."""
    seen = {}
    for q in range(256):
        K, C = W.query_shape(3, q)
        key = (_pow2(K), _pow2(C))
        if len(seen.setdefault(key, [])) < per_shape:
            seen[key].append(q)
    return sorted(q for qs in seen.values() for q in qs)


def config5_sample():
    """Serving requests whose padded shape reaches 32: K' = C' = 32, C' = 32 only, K' = 32 only."""
    want = [lambda k, c: k > 16 and c > 16, lambda k, c: k <= 16 and c > 16, lambda k, c: k > 16 and c <= 16]
    out = []
    for pred in want:
        for q in range(4000):
            K, C = W.query_shape(5, q)
            if pred(K, C):
                out.append(q)
                break
    return out


# name -> (parameter set, workload config id, query index, evaluator)
CASES = {
    "config1_toy": ("toy", 1, 0, "merged"),
    # config 1 on a 36-prime chain: the whole of Algorithm 1 without a refresh
    "config1_toy_deep": ("toy_deep", 1, 0, "merged"),
    "config2_full": ("full", 2, 0, "merged"),
    "config2_full_textbook": ("full", 2, 0, "textbook"),
}
for _q in config3_sample():
    CASES[f"config3_full_q{_q}"] = ("full", 3, _q, "merged")
for _q in config5_sample():
    CASES[f"config5_full_q{_q}"] = ("full", 5, _q, "merged")
CASES["boot13_bootstrap"] = ("p13_boot", "bootstrap", 0, "merged")
CASES["boot13_sparse"] = ("p13_boot", "bootstrap_sparse", 0, "merged")
CASES["boot13_argmax"] = ("p13_boot", "argmax_boot", 0, "merged")
CASES["boot13_packed"] = ("p13_boot", "bootstrap_packed", 0, "merged")

BOOT_SEED = 0xB007


def boot_steps(o, k_max, c_max):
    return sorted(set(o.boot_steps()) | set(argmax_rotation_steps(k_max, c_max, o.slots)),
                  key=lambda v: (v < 0, v))


def boot_input(slots):
    """The bootstrapped input: uniform slot values in [-1, 1] at scale 2^49,
    encrypted with seed 7 and lowered to level 3."""
    import numpy as np
    return np.random.default_rng(5).uniform(-1, 1, slots), 2.0**49, 7, 3


def packed_inputs(slots):
    """The window-packed case: three inputs, uniform slot values in [-1, 1]
    (generators 5, 6, 7) at scale 2^49, encrypted with seeds 7, 8, 9 and
    lowered to levels 3, 2, 3."""
    import numpy as np
    return [(np.random.default_rng(5 + j).uniform(-1, 1, slots), 2.0**49, 7 + j, 3 - j % 2) for j in range(3)]


def argmax_boot_query():
    K, C = 2, 2
    y = W.logits(9, 5, K, C)
    lo, hi = W.d_bounds(K)
    return dict(K=K, C=C, logits=y, encrypt_seed=3, refresh_seed=4, d_min=lo, d_max=hi)


def digest(arr):
    return hashlib.sha256(arr.astype("<u8").tobytes()).hexdigest()


def run_boot_case(name):
    pset, kind, _, _ = CASES[name]
    o = Oracle.from_params(W.PARAMS[pset])
    t = time.time()
    o.keygen(BOOT_SEED, boot_steps(o, 4, 4))
    tk = time.time() - t
    t = time.time()
    if kind in ("bootstrap", "bootstrap_sparse"):
        import numpy as np
        z, scale, seed, level = boot_input(o.slots)
        ct = o.lower(o.encrypt(o.encode(z, scale), scale, seed), level)
        if kind == "bootstrap":
            out = o.bootstrap(ct)
            want = z
        else:
            out = o.bootstrap_sparse(ct)
            want = np.tile(z[: o.boot_sparse], o.slots // o.boot_sparse)
        zz = o.decrypt_decode(out, o.slots)
        extra = {"max_error_log2": float(np.log2(np.abs(zz - want).max()))}
        zrec = []
    elif kind == "bootstrap_packed":
        import numpy as np
        ins = [o.lower(o.encrypt(o.encode(z, sc), sc, sd), lv) for z, sc, sd, lv in packed_inputs(o.slots)]
        outs = o.bootstrap_packed(ins)
        W_ = o.boot_sparse
        err = max(float(np.abs(o.decrypt_decode(b, o.slots)[:W_] - z[:W_]).max())
                  for b, (z, _, _, _) in zip(outs, packed_inputs(o.slots)))
        rec = {"params": pset, "kind": kind,
               "input_sha256": digest(np.concatenate([c.export().ravel() for c in ins])),
               "output_sha256": digest(np.concatenate([c.export().ravel() for c in outs])),
               "level": outs[0].level, "scale": outs[0].scale, "z": [],
               "oracle_seconds": round(time.time() - t, 1), "secret_weight": int((o.secret() != 0).sum()),
               "max_error_log2": float(np.log2(err))}
        print(f"{name}: keygen {tk:.1f} s, {rec['oracle_seconds']:.1f} s, level {rec['level']}", flush=True)
        return name, rec
    else:
        d = argmax_boot_query()
        ct = o.encrypt_logits(d["logits"], d["encrypt_seed"])
        o.reset_counters()
        out = o.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"])
        zrec = [float(v) for v in o.decrypt_decode(out, d["C"])]
        extra = {"K": d["K"], "C": d["C"], "counters": o.counters()}
    dt = time.time() - t
    rec = {"params": pset, "kind": kind, "input_sha256": digest(ct.export()), "output_sha256": digest(out.export()),
           "level": out.level, "scale": out.scale, "z": zrec, "oracle_seconds": round(dt, 1),
           "secret_weight": int((o.secret() != 0).sum())}
    rec.update(extra)
    print(f"{name}: keygen {tk:.1f} s, {dt:.1f} s, level {out.level}", flush=True)
    return name, rec


def run_case(name):
    pset, cfg, q, evaluator = CASES[name]
    if pset == "p13_boot":
        return run_boot_case(name)
    d = W.query(cfg, q)
    o = Oracle.from_params(W.PARAMS[pset])
    o.set_textbook(evaluator == "textbook")
    t = time.time()
    o.keygen(W.KEYGEN_SEED, argmax_rotation_steps(d["K"], d["C"], o.slots))
    tk = time.time() - t
    ct = o.encrypt_logits(d["logits"], d["encrypt_seed"])
    o.reset_counters()
    t = time.time()
    z = o.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"])
    dt = time.time() - t
    arr = z.export()
    zz = o.decrypt_decode(z, d["C"])
    rec = {
        "params": pset, "config": cfg, "query": q, "K": d["K"], "C": d["C"], "evaluator": evaluator,
        "input_sha256": digest(ct.export()),
        "output_sha256": digest(arr), "level": z.level, "scale": z.scale,
        "z": [float(v) for v in zz], "counters": o.counters(), "oracle_seconds": round(dt, 1),
        "secret_weight": int((o.secret() != 0).sum()),
    }
    print(f"{name}: keygen {tk:.1f} s, eval {dt:.1f} s, level {z.level}, z {zz}", flush=True)
    return name, rec


def main():
    names = sys.argv[1:] or list(CASES)
    # longest first, so the pool stays busy to the end
    cost = {"toy": 0, "toy_deep": 1, "p13_boot": -10}
    names.sort(key=lambda n: (-CASES[n][1] if CASES[n][0] == "full" else cost.get(CASES[n][0], 0)))
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    workers = int(os.environ.get("GOLDEN_WORKERS", "8"))
    with ProcessPoolExecutor(workers) as ex:
        for name, rec in ex.map(run_case, names):
            out[name] = rec
            with open(OUT, "w") as f:
                json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
