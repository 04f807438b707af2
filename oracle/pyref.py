"""Pure-Python re-statement of the oracle's definitions, for tiny inputs.

TEST INFRASTRUCTURE. Written separately from abc_oracle.c and used only to
cross-check it: Philox4x32-10 on Python integers, the prior draw in exact
rational arithmetic, the model of Sec. 2.1 with Python ints for counts and
floats (IEEE double) for rates. Slow by design.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox(ctr, key, rounds=10):
    """Philox4x32 (Salmon et al., SC'11): rounds of two 32x32->64 products,
    the word permutation and XOR with the key, the key bumped by the Weyl
    constants between rounds."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK, (p0 >> 32) ^ c3 ^ k1, p0 & MASK)
    return c0, c1, c2, c3


def words(seed, domain, series, sample, day, block):
    key = (seed & MASK, seed >> 32)
    ctr = (sample & MASK, sample >> 32, series, (day << 8) | (domain << 4) | block)
    return philox(ctr, key)


def _round_to_f32(x: Fraction) -> float:
    """Round an exact rational to the nearest binary32 (ties to even)."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    x = abs(x)
    e = math.floor(math.log2(x.numerator) - math.log2(x.denominator))
    # fix possible off-by-one of the float log estimate
    while Fraction(2) ** e > x:
        e -= 1
    while Fraction(2) ** (e + 1) <= x:
        e += 1
    e = max(e, -126)
    scale = Fraction(2) ** (e - 23)
    q = x / scale
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return sign * float(n * scale)


def prior_theta(seed, domain, series, sample, lo, hi):
    w = list(words(seed, domain, series, sample, 0, 0)) + list(words(seed, domain, series,
                                                                     sample, 0, 1))
    out = []
    for k in range(8):
        u = Fraction(w[k] >> 8, 1 << 24)
        lo_k = Fraction(float(np.float32(lo[k])))
        width = Fraction(_round_to_f32(Fraction(float(np.float32(hi[k]))) - lo_k))
        out.append(_round_to_f32(width * u + lo_k))
    return np.array(out, dtype=np.float32)


def normals(seed, domain, series, sample, day):
    w0, w1, w2, w3 = words(seed, domain, series, sample, day, 0)
    f = [w0 >> 11, w1 >> 11, w2 >> 11, w3 >> 11,
         ((w0 & 0x7FF) << 10) | (w1 & 0x3FF), ((w2 & 0x7FF) << 10) | (w3 & 0x3FF)]
    u = [(x + 0.5) / (1 << 21) for x in f]
    r = [math.sqrt(-2.0 * math.log(u[0])), math.sqrt(-2.0 * math.log(u[2])),
         math.sqrt(-2.0 * math.log(u[4]))]
    tp = 2.0 * math.pi
    return [r[0] * math.cos(tp * u[1]), r[0] * math.sin(tp * u[1]),
            r[1] * math.cos(tp * u[3]), r[1] * math.sin(tp * u[3]),
            r[2] * math.cos(tp * u[5])]


def trajectory(theta, P, T, A0=100, R0=0, D0=0, seed=0, domain=1, series=0, sample=0,
               noise_scale=1.0, noise_mode=0, obs=None, dist_mode=0):
    a0, al, n, be, ga, de, et, ka = (float(x) for x in np.asarray(theta, dtype=np.float32))
    A, R, D, Ru = int(A0), int(R0), int(D0), 0
    I = math.floor(ka * A0)
    S = int(P) - (A + R + D + I)
    rows = [(S, I, A, R, D, Ru)]
    acc = 0.0

    def draw(h, z, avail):
        sd = noise_scale * (math.sqrt(h) if noise_mode == 0 else math.sqrt(math.sqrt(h)))
        f = math.floor(h + sd * z)
        return min(max(f, 0), avail)

    for t in range(1, T + 1):
        M = float(A + R + D)
        g = a0 + al / (1.0 + M ** n)
        h = (g * S * I / P, ga * I, be * A, de * A, be * et * I)
        z = normals(seed, domain, series, sample, t)
        n1 = draw(h[0], z[0], S)
        n2 = draw(h[1], z[1], I)
        n3 = draw(h[2], z[2], A)
        n4 = draw(h[3], z[3], A - n3)
        n5 = draw(h[4], z[4], I - n2)
        S -= n1
        I += n1 - n2 - n5
        A += n2 - n3 - n4
        R += n3
        D += n4
        Ru += n5
        rows.append((S, I, A, R, D, Ru))
        if obs is not None:
            for c, X in enumerate((A, R, D)):
                O = int(obs[c][t - 1])
                d = (math.log1p(X) - math.log1p(O)) if dist_mode == 0 else float(X - O)
                acc += d * d
    return np.array(rows, dtype=np.int64), (math.sqrt(acc) if obs is not None else None)
