"""Seeded synthetic workloads for the encrypted Argmax.

Shared by the GPU path's tests/bench and by the CPU oracle's tests.  It holds
no CKKS or Argmax arithmetic: only parameter sets, seeds, shapes and logits.

The paper measures on GLUE/AdvGLUE, GSM8K/MultiArith and ImageNet/CIFAR with
trained models (Sec. 4); none of that is needed for the Argmax, whose input is
a K x C block of per-prompt class scores.  These generators stand in for it:
i.i.d. N(0,1) logits, clipped at +-6, drawn from numpy's PCG64 seeded by
SeedSequence([config_id, query]).
"""
import numpy as np

# CKKS parameter sets.  n_q chain primes of q_bits, n_p special primes below
# 2^p_bits (alpha = n_p primes per key-switch digit), scale 2^log_scale.
# refresh_level: level a refreshed ciphertext comes back at (the paper's
# bootstrapping leaves K = 14 levels, Sec. 4.1); absent = the top level.
PARAMS = {
    # N=2^13, 8 x 30-bit primes + 1 special prime, scale 2^30 (correctness only)
    "toy": dict(log_n=13, n_q=8, q_bits=30, n_p=1, p_bits=51, log_scale=30, dg=2, df=2, min_level=1),
    # N=2^16, 24 x ~50-bit primes, 8 special primes (dnum = 3 digits), scale 2^50
    "full": dict(log_n=16, n_q=24, q_bits=50, n_p=8, p_bits=51, log_scale=50, dg=2, df=2, min_level=1,
                 refresh_level=14),
    # N=2^16 with 3 special primes (dnum = 8 digits)
    "full_a3": dict(log_n=16, n_q=24, q_bits=50, n_p=3, p_bits=51, log_scale=50, dg=2, df=2, min_level=1,
                    refresh_level=14),
    # config 1 without any refresh: the whole of Algorithm 1 for C' = 2 on a
    # 36-prime chain (alpha = 4, dnum = 9), non-interactively
    "toy_deep": dict(log_n=13, n_q=36, q_bits=30, n_p=4, p_bits=51, log_scale=30, dg=2, df=2, min_level=1),
    # small parameter sets for fast unit tests
    "tiny": dict(log_n=10, n_q=8, q_bits=40, n_p=2, p_bits=51, log_scale=40, dg=2, df=2, min_level=1),
    # tiny with refreshes re-encrypting below the top level
    "tiny_r6": dict(log_n=10, n_q=8, q_bits=40, n_p=2, p_bits=51, log_scale=40, dg=2, df=2, min_level=1,
                    refresh_level=6),
    "mini": dict(log_n=11, n_q=10, q_bits=45, n_p=4, p_bits=51, log_scale=45, dg=2, df=2, min_level=1),
    # Bootstrapping sets: sparse secret of expected weight h; EvalMod on
    # |t / q_0| <= boot_K + 1 with a degree-boot_deg Chebyshev interpolant and
    # boot_r double angles; q_0 / T_b = 2^boot_ratio; boot_groups levels for each
    # linear transform; boot_refresh = 1 makes every refresh a bootstrap;
    # boot_sparse = n adds the sparse-slot bootstrap of slots [0, n), which
    # refreshes of a single query take (it reads slots [0, 2C') only).
    # 2 * 3 + 6 + 3 = 15 levels on N = 2^10 (a bootstrapped ciphertext has 10 left)
    "tiny_boot": dict(log_n=10, n_q=26, q_bits=50, n_p=8, p_bits=51, log_scale=50, dg=2, df=2, min_level=1,
                      h=64, boot_K=12, boot_r=3, boot_deg=31, boot_ratio=8, boot_groups=3, boot_refresh=1,
                      boot_sparse=32),
    # the tiny_boot chain at N = 2^13: the two-pass NTT, the fused ModUp /
    # inner-product kernels and baby-step giant-step groups of n1 = 8 baby
    # steps, as at N = 2^16 (a bootstrapped ciphertext has 10 levels left)
    "p13_boot": dict(log_n=13, n_q=26, q_bits=50, n_p=8, p_bits=51, log_scale=50, dg=2, df=2, min_level=1,
                     h=64, boot_K=12, boot_r=3, boot_deg=31, boot_ratio=8, boot_groups=3, boot_refresh=1,
                     boot_sparse=32),
    # L = 35 chain primes as in the paper (Sec. 4.1); 2 * 3 + 6 + 4 = 16 levels,
    # a bootstrapped ciphertext has 18 left.  boot_sparse: the sparse-slot
    # bootstrap keeps slots [0, 64), enough for a single query up to C' = 32
    "full_boot": dict(log_n=16, n_q=35, q_bits=50, n_p=12, p_bits=51, log_scale=50, dg=2, df=2, min_level=1,
                      h=192, boot_K=24, boot_r=4, boot_deg=31, boot_ratio=8, boot_groups=3, boot_refresh=1,
                      boot_sparse=64),
    # The paper's budget (Sec. 4.1): N = 2^16, L = 35 chain primes, log QP <=
    # 1763 bits, 14 levels for bootstrapping.  35 primes of ~47 bits and 2
    # special primes below 2^51 (dnum 18) make log QP = 1747; 2 + 2 groups,
    # degree 31 and 4 double angles make 2 * 2 + 6 + 4 = 14 levels, leaving a
    # bootstrapped ciphertext 20 levels.
    "full_boot128": dict(log_n=16, n_q=35, q_bits=47, n_p=2, p_bits=51, log_scale=47, dg=2, df=2, min_level=1,
                         h=192, boot_K=24, boot_r=4, boot_deg=31, boot_ratio=8, boot_groups=2, boot_refresh=1,
                         boot_sparse=64),
}

CLIP = 6.0
KEYGEN_SEED = 0x5EC0_5EED_0000_0001


def rng(config_id, query):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config_id), int(query)])))


def logits(config_id, query, K, C, min_margin=None):
    """K x C logits, N(0,1) clipped to +-6; redrawn until the top-2 margin of the
    prompt sum is at least min_margin (when given)."""
    g = rng(config_id, query)
    while True:
        y = np.clip(g.standard_normal((K, C)), -CLIP, CLIP)
        if min_margin is None or C < 2:
            return y
        s = np.sort(y.sum(axis=0))
        if s[-1] - s[-2] >= min_margin:
            return y


def d_bounds(K):
    """Public normalisation bounds: the prompt sum of clipped logits lies in [-6K, 6K]."""
    return -CLIP * K, CLIP * K


def query_seeds(config_id, query):
    """(encrypt_seed, refresh_seed) as uint64 values."""
    g = rng(1000 + int(config_id), query)
    s = g.integers(0, 2**63, size=2, dtype=np.int64)
    return int(s[0]), int(s[1])


def query_shape(config_id, query):
    """(K, C) of a query for each workload."""
    if config_id == 1:
        return 4, 2
    if config_id == 2:
        return 8, 4
    if config_id == 3:
        g = rng(3, query)
        return int(g.integers(3, 17)), int(g.integers(2, 15))
    if config_id == 5:
        g = rng(5, query)
        return int(g.integers(4, 33)), int(g.integers(2, 21))
    raise ValueError(config_id)


def query(config_id, q):
    """Everything that defines one query: shape, logits, seeds and bounds."""
    K, C = query_shape(config_id, q)
    y = logits(config_id, q, K, C, min_margin=0.05 if config_id == 2 else None)
    enc, ref = query_seeds(config_id, q)
    dmin, dmax = d_bounds(K)
    return dict(K=K, C=C, logits=y, encrypt_seed=enc, refresh_seed=ref, d_min=dmin, d_max=dmax)


def poisson_arrivals(qps, n, seed=(5, 0)):
    """Arrival times (seconds) of n requests with exponential gaps at rate qps."""
    g = rng(*seed)
    return np.cumsum(g.exponential(1.0 / qps, size=n))


def random_rotation_steps(n, slots, seed=(4, 0)):
    """n rotation amounts uniform in [1, slots) for the rotation microbenchmark."""
    g = rng(*seed)
    return [int(v) for v in g.integers(1, slots, size=n)]
