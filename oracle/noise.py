"""Noise model of the encrypted Argmax (test infrastructure; see oracle/__init__.py).

Algorithm 1 (Sec. 3.2) in FP64, as in sim.t1_argmax, with the rounding noise
of every RNS-CKKS step (Sec. 2.2) added where the encrypted evaluation incurs
it.  It derives how far two evaluations of the same query may drift apart
and how far either may drift from the noiseless result, for the two
evaluators the oracle implements:

  merged    a product is relinearised and rescaled in one division by P q_l
            (the approximate conversion from the n_p + 1 primes of P q_l
            rounds), the degree-1 addend of a Sign polynomial's last sum and
            the (a+b)/2 of Max are added before that one division;
  textbook  tensor, relinearise (hybrid key switch), rescale, each product on
            its own; every constant combination rescaled once.

Per-step noise.  A step that rounds a ciphertext's coefficients leaves the
decrypted message with e = r0 + r1 s, the r being the step's rounding
residues (independent, variance V per coefficient), so Var(e_k) = V (1 + h)
with h the number of nonzero secret coefficients.  Decoding divides by the
scale Delta and sums N coefficients per slot with unit-modulus weights, so a
slot's real part gets variance (N/2) Var(e_k) / Delta^2.  The residues:

  rescale by q_l (centred remainder)           V = 1/12
  key switch: ModDown from n_p special primes  V = (n_p + 1)/12   (rounding plus
                                                the integer overflow of the
                                                centred conversion)
              plus the key's error over P       dnum N D^2 sigma_e^2 / (3 P^2)
                                                (D: a digit's modulus, digits
                                                lifted to [0, D); not times s)
  merged relinearise-and-rescale over P q_l    V = (n_p + 2)/12
  refresh stand-in: fresh encryption error     Var = sigma_e^2 (not times s)

with sigma_e^2 = 10.5 (centred binomial, eta = 21).  A textbook product's own
key switch is divided by q_l by its rescale and left out; so are the roundings
of the integer constants (relative 2^-log_scale).  Every scale is taken as
Delta (each prime is within a few parts in 2^12 of it).

Two evaluators of one query share every step before the first Sign
polynomial (prompt sum, Eq. 5, duplication, the first QuickMax rotation) and
the refresh errors (same seeds); every later rounding residue depends on
their differing inputs and is drawn independently.  Monte Carlo over such
pairs gives the spread of z_merged - z_textbook per slot.

The slot vector is cut to S = 2^ceil(log2 max(K'C', 2C')) slots: every value
Algorithm 1 reads for the outputs [0, C) lies in [0, S), and the masked tail
that the duplication rotates in is zero (plus noise of the same law) either
way.
"""
import numpy as np

from .sim import F4, G4, _pow2ceil, odd_poly

SIGMA_E2 = 10.5


class _Val:
    __slots__ = ("v", "level")

    def __init__(self, v, level):
        self.v = v
        self.level = level


class _NoisyArgmax:
    def __init__(self, mode, prm, h, S, rng_common, rng_own, refresh_noise):
        assert mode in ("merged", "textbook")
        self.mode = mode
        N = 1 << prm["log_n"]
        n_q, n_p = prm["n_q"], prm["n_p"]
        delta = 2.0 ** prm["log_scale"]
        dnum = -(-n_q // n_p)
        base = (N / 2.0) / delta**2
        # key-switch error over P relative to one digit's modulus: D / P
        d_over_p2 = 2.0 ** (2 * (prm["q_bits"] * n_p - prm["p_bits"] * n_p))
        self.sd = dict(
            ks=np.sqrt(base * ((1 + h) * (n_p + 1) / 12.0 + dnum * N * d_over_p2 * SIGMA_E2 / 3.0)),
            mrr=np.sqrt(base * (1 + h) * (n_p + 2) / 12.0),
            rs=np.sqrt(base * (1 + h) / 12.0),
            enc=np.sqrt(base * SIGMA_E2),
        )
        self.top = n_q - 1
        rl = prm.get("refresh_level", 0)
        self.refresh_level = rl if 0 < rl < n_q else self.top
        self.min_level = prm.get("min_level", 1)
        self.dg, self.df = prm.get("dg", 2), prm.get("df", 2)
        self.S = S
        self.rc, self.ro = rng_common, rng_own
        self.refresh_noise = refresh_noise
        self.n_refresh = 0
        self.common = True

    def _n(self, kind):
        rng = self.rc if self.common else self.ro
        return rng.normal(0.0, self.sd[kind], self.S)

    def _refresh(self, x, need):
        if x.level - need >= self.min_level:
            return x
        if self.refresh_level - need < self.min_level:
            raise ValueError("modulus chain too short for one unit")
        v = x.v + self.refresh_noise[self.n_refresh]
        self.n_refresh += 1
        return _Val(v, self.refresh_level)

    def _rot(self, x, r):
        return _Val(np.roll(x.v, -r) + self._n("ks"), x.level)

    def _poly(self, x, coef):
        self.common = False
        k1, k3, k5, k7, k9 = coef
        v = x.v
        if self.mode == "merged":
            x2 = v * v + self._n("mrr")
            x3 = x2 * v + self._n("mrr")
            x4 = x2 * x2 + self._n("mrr")
            x8 = x4 * x4 + self._n("mrr")
            A = k1 * v + k3 * x3
            B = k5 * v + k7 * x3 + self._n("rs")
            Cc = k9 * v + self._n("rs")
            p = x4 * B + x8 * Cc + A + self._n("mrr")
        else:
            x2 = v * v + self._n("rs")
            x3 = x2 * v + self._n("rs")
            x4 = x2 * x2 + self._n("rs")
            x8 = x4 * x4 + self._n("rs")
            B = k5 * v + k7 * x3 + self._n("rs")
            Cc = k9 * v + self._n("rs")
            A = k1 * v + k3 * x3 + self._n("rs")
            t = x4 * B + self._n("rs")
            u = x8 * Cc + self._n("rs")
            p = t + u + A
        return _Val(p, x.level - 4)

    def _sign(self, x, gain, extra):
        total = self.dg + self.df
        for i in range(total):
            last = i == total - 1
            x = self._refresh(x, 4 + (extra if last else 0))
            coef = np.array(G4 if i < self.dg else F4) * (gain if last else 1.0)
            x = self._poly(x, coef)
        return x

    def _sign_level(self, level, extra):
        # the level the last polynomial lands on (the refresh decisions planned ahead)
        total = self.dg + self.df
        for i in range(total):
            need = 4 + (extra if i == total - 1 else 0)
            if level - need < self.min_level:
                level = self.refresh_level
            level -= 4
        return level

    def _max(self, a, b):
        ld = min(a.level, b.level)
        d = _Val(a.v - b.v, ld)
        s = a.v + b.v
        lp = min(ld, self._sign_level(ld, 1))
        sg = self._sign(d, 0.5, 1)
        if self.mode == "merged":
            out = d.v * sg.v + 0.5 * s + self._n("mrr")
        else:
            out = (d.v * sg.v + self._n("rs")) + (0.5 * s + self._n("rs"))
        return _Val(out, lp - 1)

    def run(self, logits, d_min, d_max):
        logits = np.asarray(logits, dtype=np.float64)
        K, C = logits.shape
        Kp, Cp = _pow2ceil(K), _pow2ceil(C)
        S = self.S
        y = np.zeros(S)
        for k in range(K):
            y[k * Cp:k * Cp + C] = logits[k]
        x = _Val(y + self._n("enc"), self.top)
        i = 1
        while i < Kp:
            r = self._rot(x, Cp * i)
            x = _Val(x.v + r.v, x.level)
            i <<= 1
        x = self._refresh(x, 1)
        mask = np.zeros(S)
        mask[:C] = 1.0
        x = _Val(mask * (x.v - d_min) / (d_max - d_min) + self._n("rs"), x.level - 1)
        r = self._rot(x, S - Cp)
        ydup = _Val(x.v + r.v, x.level)
        ym = ydup
        i = 1
        while i < Cp:
            ym = self._refresh(ym, 1)
            r = self._rot(ym, i)
            ym = self._max(r, ym)
            i <<= 1
        d = _Val(ydup.v - ym.v, min(ydup.level, ym.level))
        z = self._sign(d, 1.0, 0)
        return z.v[:C] + 1.0


def argmax_noise_samples(logits, d_min, d_max, prm, h, n_pairs=200, seed=0):
    """z[:C] of n_pairs noisy runs of Algorithm 1 per evaluator, pair i of the
    two evaluators sharing the common noise: {'merged': [n, C], 'textbook': [n, C]}."""
    logits = np.asarray(logits, dtype=np.float64)
    K, C = logits.shape
    Kp, Cp = _pow2ceil(K), _pow2ceil(C)
    S = min((1 << prm["log_n"]) // 2, _pow2ceil(max(Kp * Cp, 2 * Cp, 2)))
    out = {"merged": [], "textbook": []}
    root = np.random.SeedSequence([int(seed), K, C])
    for pair_seed in root.spawn(n_pairs):
        s_common, s_ref, s_m, s_t = pair_seed.spawn(4)
        probe = _NoisyArgmax("merged", prm, h, S, None, None, None)
        rref = np.random.default_rng(s_ref)
        refresh_noise = [rref.normal(0.0, probe.sd["enc"], S) for _ in range(256)]
        for mode, s_own in (("merged", s_m), ("textbook", s_t)):
            sim = _NoisyArgmax(mode, prm, h, S, np.random.default_rng(s_common), np.random.default_rng(s_own),
                               refresh_noise)
            out[mode].append(sim.run(logits, d_min, d_max))
    return {k: np.array(v) for k, v in out.items()}


def noiseless(logits, d_min, d_max, prm):
    """The same data flow with every noise term zero (equals sim.t1_argmax[:C])."""
    logits = np.asarray(logits, dtype=np.float64)
    K, C = logits.shape
    Kp, Cp = _pow2ceil(K), _pow2ceil(C)
    S = min((1 << prm["log_n"]) // 2, _pow2ceil(max(Kp * Cp, 2 * Cp, 2)))
    sim = _NoisyArgmax("merged", prm, 0, S, None, None, [np.zeros(S)] * 256)
    sim.sd = {k: 0.0 for k in sim.sd}

    class _Zero:
        @staticmethod
        def normal(loc, scale, size):
            return np.zeros(size)

    sim.rc = sim.ro = _Zero()
    return sim.run(logits, d_min, d_max)


__all__ = ["argmax_noise_samples", "noiseless", "odd_poly"]
