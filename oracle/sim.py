"""FP64 tiers of the oracle (test infrastructure; see oracle/__init__.py).

t0_*  the plain definition: argmax of the prompt sum (Sec. 2.3, prompt ensembling;
      Sec. 3.2, Eq. 1: one-hot at the largest entry).
t1_*  Algorithm 1 (Sec. 3.2) in FP64 on the full real slot vector, with the
      composite polynomial Sign (Eq. 4), Max (Eq. 6) and normalisation (Eq. 5).
      It follows the same data flow as the encrypted evaluation, rotations
      included, so it shows the approximation error without encryption noise.
"""
import numpy as np

# f_4 and g_4 (odd coefficients of x, x^3, x^5, x^7, x^9); the paper prints
# neither, only "degree 9".  f_4 is the closed form sum_{i<=4} C(2i,i) 4^-i
# x (1-x^2)^i; g_4 is Cheon-Kim-Kim's degree-9 g (ASIACRYPT 2020).
F4 = np.array([315.0, -420.0, 378.0, -180.0, 35.0]) / 128.0
G4 = np.array([5850.0, -34974.0, 97015.0, -113492.0, 46623.0]) / 1024.0


def odd_poly(coef, x):
    """sum_k coef[k] x^(2k+1)."""
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    acc = np.zeros_like(x) + coef[-1]
    for c in coef[-2::-1]:
        acc = acc * x2 + c
    return acc * x


def sign_composite(x, dg=2, df=2, f=F4, g=G4):
    """Sign(x) ~ f^df(g^dg(x)) on [-1, 1]  (Eq. 4)."""
    y = np.asarray(x, dtype=np.float64)
    for _ in range(dg):
        y = odd_poly(g, y)
    for _ in range(df):
        y = odd_poly(f, y)
    return y


def sign_threshold(dg=2, df=2, tol=1e-4, lo=-20.0, points=200001):
    """Smallest eps (as log2) such that |S(x) - 1| <= tol on [eps, 1] (grid in log2 x)."""
    e = np.linspace(lo, 0.0, points)
    x = np.exp2(e)
    bad = np.abs(sign_composite(x, dg, df) - 1.0) > tol
    if not bad.any():
        return lo
    return float(e[np.nonzero(bad)[0].max() + 1]) if bad.nonzero()[0].max() + 1 < points else 0.0


def t0_argmax(logits):
    """Definition: y* = sum over prompts; index of the largest (lowest index on ties)."""
    y = np.asarray(logits, dtype=np.float64).sum(axis=0)
    idx = int(np.argmax(y))
    srt = np.sort(y)
    margin = float(srt[-1] - srt[-2]) if len(y) > 1 else float("inf")
    return idx, y, margin


def _pow2ceil(v):
    return 1 << max(0, int(v - 1).bit_length())


def t1_argmax(logits, d_min, d_max, slots, dg=2, df=2, exact_sign=False, return_all=False):
    """Algorithm 1 on the real slot vector.  RotL(y, r)[j] = y[(j + r) mod slots]."""
    logits = np.asarray(logits, dtype=np.float64)
    K, C = logits.shape
    Kp, Cp = _pow2ceil(K), _pow2ceil(C)
    sgn = np.sign if exact_sign else (lambda v: sign_composite(v, dg, df))
    y = np.zeros(slots)
    for k in range(K):
        y[k * Cp:k * Cp + C] = logits[k]
    i = 1
    while i < Kp:                                  # sum over prompts by doubling
        y = y + np.roll(y, -Cp * i)
        i <<= 1
    mask = np.zeros(slots)
    mask[:C] = 1.0
    y = mask * (y - d_min) / (d_max - d_min)       # Eq. 5
    y = y + np.roll(y, Cp)                          # line 2: y + RotR(y, n)
    ym = y.copy()
    i = 1
    while i < Cp:                                  # line 3: QuickMax
        r = np.roll(ym, -i)
        ym = (r + ym) / 2 + (r - ym) / 2 * sgn(r - ym)   # Eq. 6
        i <<= 1
    d = y - ym                                     # line 4
    z = sgn(d) + 1.0                               # lines 5-6, Eq. 2
    if return_all:
        return z, dict(y=y, ymax=ym)
    return z[:C]


def packed_shape(shapes):
    """(K', C', block size) of a packed group: the largest padded shape, blocks of max(K'C', 2C')."""
    Kp = max(_pow2ceil(K) for K, _ in shapes)
    Cp = max(_pow2ceil(C) for _, C in shapes)
    return Kp, Cp, max(Kp * Cp, 2 * Cp)


def t1_argmax_packed(blocks, slots, dg=2, df=2, exact_sign=False):
    """Algorithm 1 on a packed slot vector (Sec. 3.2: several Argmax inputs in one
    ciphertext).  blocks: list of (logits K_b x C_b, d_min_b, d_max_b); query b
    sits at slot b*B + k*C' + c.  Returns each block's z[:C_b]."""
    shapes = [np.asarray(l).shape for l, _, _ in blocks]
    Kp, Cp, B = packed_shape(shapes)
    assert len(blocks) * B <= slots
    sgn = np.sign if exact_sign else (lambda v: sign_composite(v, dg, df))
    y = np.zeros(slots)
    shift = np.zeros(slots)
    mask = np.zeros(slots)
    for b, (lg, lo, hi) in enumerate(blocks):
        lg = np.asarray(lg, dtype=np.float64)
        K, C = lg.shape
        for k in range(K):
            y[b * B + k * Cp:b * B + k * Cp + C] = lg[k]
        shift[b * B:b * B + C] = -lo
        mask[b * B:b * B + C] = 1.0 / (hi - lo)
    i = 1
    while i < Kp:
        y = y + np.roll(y, -Cp * i)
        i <<= 1
    y = mask * (y + shift)                          # Eq. 5 per block
    y = y + np.roll(y, Cp)
    ym = y.copy()
    i = 1
    while i < Cp:
        r = np.roll(ym, -i)
        ym = (r + ym) / 2 + (r - ym) / 2 * sgn(r - ym)
        i <<= 1
    z = sgn(y - ym) + 1.0
    return [z[b * B:b * B + s[1]] for b, s in enumerate(shapes)]


def t1_argmax_phoenix(logits, d_min, d_max, slots, dg=2, df=2, exact_sign=False):
    """The comparison path (Phoenix, Sec. 3.2) on the real slot vector: prompt sum
    and Eq. 5 as in Algorithm 1, then s = sum_{i<C} Sign(y - RotL(y, i)) with y
    duplicated at offset C, and z = (Sign((s - (C-2)) / (2C-3)) + 1) / 2."""
    logits = np.asarray(logits, dtype=np.float64)
    K, C = logits.shape
    Kp, Cp = _pow2ceil(K), _pow2ceil(C)
    sgn = np.sign if exact_sign else (lambda v: sign_composite(v, dg, df))
    y = np.zeros(slots)
    for k in range(K):
        y[k * Cp:k * Cp + C] = logits[k]
    i = 1
    while i < Kp:
        y = y + np.roll(y, -Cp * i)
        i <<= 1
    mask = np.zeros(slots)
    mask[:C] = 1.0
    y = mask * (y - d_min) / (d_max - d_min)
    y = y + np.roll(y, C)
    s = np.zeros(slots)
    for i in range(1, C):
        s = s + sgn(y - np.roll(y, -i))
    x = (s - (C - 2)) / (2 * C - 3)
    z = 0.5 * sgn(x) + 0.5
    return z[:C]


def decoded_index(z):
    return int(np.argmax(np.asarray(z)))
