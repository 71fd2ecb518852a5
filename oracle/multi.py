"""CPU oracle for multi-allelic markers (genotype classes 0..l, l >= 2).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite
may import it.  Plain Python with exact integers, for small cases.

The statistic is eq. (2) divided by the tie factor (Handling tied data), with
one group per genotype class present among the kept samples; the p-value is
the chi-square tail with df = (non-empty classes - 1) (P-value calculation),
for any df.  A sample is kept when its expression value is not NaN and its
genotype code is one of 0..l; the ranks are taken over the kept samples
(Handling missing values).
"""
import math
import struct
from fractions import Fraction

import numpy as np


def chi2_tail(H, df):
    """Upper tail of the chi-square distribution with df degrees of freedom
    at H, from the closed forms of the regularised upper incomplete gamma
    Q(df/2, H/2): an exponential times a finite sum for even df, plus erfc
    for odd df."""
    if df <= 0:
        return 1.0
    x = 0.5 * float(H)
    if df % 2 == 0:
        term, total = 1.0, 1.0
        for k in range(1, df // 2):
            term *= x / k
            total += term
        return math.exp(-x) * total
    total = math.erfc(math.sqrt(x))
    if df > 1:
        # sum_{k=1}^{(df-1)/2} x^(k-1/2) / Gamma(k + 1/2)
        term = math.sqrt(x) / math.gamma(1.5)
        s = term
        for k in range(2, (df - 1) // 2 + 1):
            term *= x / (k - 0.5)
            s += term
        total += math.exp(-x) * s
    return total


def _bits(d):
    return struct.unpack("<q", struct.pack("<d", d))[0]


def _double(b):
    return struct.unpack("<d", struct.pack("<q", b))[0]


def threshold(p_c, df):
    """Largest double h >= 0 with chi2_tail(h, df) >= p_c (p_c in (0, 1])."""
    if not (0.0 < p_c <= 1.0) or df < 1:
        return float("nan")
    lo, hi = 0, _bits(float("inf"))        # chi2_tail(lo) >= p_c > chi2_tail(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if chi2_tail(_double(mid), df) >= p_c:
            lo = mid
        else:
            hi = mid
    return _double(lo)


def one_pair(x, g, n_classes):
    """One trait row x (K,) float and genotype row g (K,) int with classes
    0..n_classes-1 -> dict(H, p, df, n, s2, tiesum, kobs); s2 holds the
    groups' sums of doubled midranks over the kept samples."""
    x = np.asarray(x, dtype=np.float32)
    g = np.asarray(g).astype(np.int64)
    keep = np.flatnonzero(~np.isnan(x) & (g >= 0) & (g < n_classes))
    vals = x[keep].astype(np.float64)
    kp = len(keep)
    # doubled midrank of each kept sample by counting: 2 #below + #equal + 1
    less = (vals[None, :] < vals[:, None]).sum(axis=1)
    eq = (vals[None, :] == vals[:, None]).sum(axis=1)
    a2 = [int(v) for v in 2 * less + eq + 1]
    tiesum = 0
    for v in set(vals.tolist()):
        t = int((vals == v).sum())
        tiesum += t ** 3 - t
    n = [0] * n_classes
    s2 = [0] * n_classes
    for j, k in enumerate(keep):
        c = int(g[k])
        n[c] += 1
        s2[c] += a2[j]
    nonempty = sum(1 for c in n if c > 0)
    df = nonempty - 1 if nonempty > 0 else 0
    E = kp ** 3 - kp - tiesum
    if df <= 0 or kp < 2 or E <= 0:
        H = 0.0
    else:
        # doubled ranks centred at K'+1: D_c = s2_c - n_c (K'+1)
        f = sum(Fraction((s2[c] - n[c] * (kp + 1)) ** 2, n[c]) for c in range(n_classes)
                if n[c])
        H = float(Fraction(3 * (kp - 1)) * f / E)
    p = chi2_tail(H, df) if df > 0 else 1.0
    return dict(H=H, p=p, df=df, n=n, s2=s2, tiesum=tiesum, kobs=kp)


def scan(expr, geno, n_classes, p_c=None):
    """Every pair: H, p (T, M) and, with p_c, the hits (trait, snp) with
    H > threshold(p_c, df) in (trait, snp) order."""
    T, M = expr.shape[0], geno.shape[0]
    H = np.zeros((T, M))
    p = np.ones((T, M))
    hits = []
    for t in range(T):
        for m in range(M):
            o = one_pair(expr[t], geno[m], n_classes)
            H[t, m], p[t, m] = o["H"], o["p"]
            if p_c is not None and o["df"] > 0 and o["H"] > threshold(p_c, o["df"]):
                hits.append((t, m))
    return dict(H=H, p=p, hits=hits)
