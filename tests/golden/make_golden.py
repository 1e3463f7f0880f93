"""Write tests/golden/argmax_digests.json from the CPU oracle only.

For each case the oracle encrypts the seeded logits, evaluates the encrypted
Argmax (Algorithm 1) and records: the SHA-256 of the output ciphertext in the
coefficient domain (canonical residues, uint64 little-endian, [2][level+1][N]),
its level and scale, the decrypted z and the operation counts.  The GPU parity
test recomputes the same digest from the HIP path.

Cases: config 1 (toy N=2^13, 8 x 30-bit primes, K=4, C=2; and on 36 primes,
alpha = 4, with no refresh at all) and config 2
(N=2^16, 24 x 50-bit primes, dnum 3, K=8, C=4, margin >= 0.05), plus one
config-3 query.  Run from the repository root: python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workload as W  # noqa: E402
from oracle.ckks import Oracle, argmax_rotation_steps  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "argmax_digests.json")

CASES = [
    # name, parameter set, workload config id, query index, rotation keys for (k_max, c_max)
    ("config1_toy", "toy", 1, 0, (4, 2)),
    # config 1 on a 36-prime chain: the whole of Algorithm 1 without a refresh
    ("config1_toy_deep", "toy_deep", 1, 0, (4, 2)),
    ("config2_full", "full", 2, 0, (16, 14)),
    ("config3_full_q0", "full", 3, 0, (16, 14)),
]


def digest(arr):
    return hashlib.sha256(arr.astype("<u8").tobytes()).hexdigest()


def run_case(name, pset, cfg, q, kc, orc_cache):
    o = orc_cache.get(pset)
    if o is None:
        o = Oracle.from_params(W.PARAMS[pset])
        t = time.time()
        o.keygen(W.KEYGEN_SEED, argmax_rotation_steps(*kc, o.slots))
        print(f"[{pset}] keygen {time.time() - t:.1f} s", flush=True)
        orc_cache[pset] = o
    d = W.query(cfg, q)
    ct = o.encrypt_logits(d["logits"], d["encrypt_seed"])
    o.reset_counters()
    t = time.time()
    z = o.eval_argmax(ct, d["K"], d["C"], d["d_min"], d["d_max"], d["refresh_seed"])
    dt = time.time() - t
    arr = z.export()
    zz = o.decrypt_decode(z, d["C"])
    rec = {
        "params": pset, "config": cfg, "query": q, "K": d["K"], "C": d["C"],
        "input_sha256": digest(ct.export()),
        "output_sha256": digest(arr), "level": z.level, "scale": z.scale,
        "z": [float(v) for v in zz], "counters": o.counters(), "oracle_seconds": round(dt, 1),
    }
    print(f"{name}: {dt:.1f} s, level {z.level}, z {zz}", flush=True)
    return rec


def main():
    names = sys.argv[1:] or [c[0] for c in CASES]
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    cache = {}
    for case in CASES:
        if case[0] in names:
            out[case[0]] = run_case(*case, cache)
            with open(OUT, "w") as f:
                json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
