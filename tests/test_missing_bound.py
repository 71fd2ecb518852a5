"""The bound behind the re-rank filter for SNPs with missing genotypes
(sample exclusion with re-ranking over the rest, section 2), checked by
brute force on small inputs with heavy ties.

Removing missing sample q shifts the centred rank sum of group i by
-s_i(q), s_i(q) = #{kept k in group i above q} - #{kept k in group i below q};
from q's doubled midrank a_q alone, at most (a_q - 2) / 2 samples lie below q
and at most K - a_q / 2 above it, so s_i(q) lies in
[-min(N_i, (a_q - 2) // 2), min(N_i, K - (a_q + 1) // 2)].  Counting q's tie
partners too, 2 #below + (t_q - 1) = a_q - 2 and 2 #above + (t_q - 1) = 2K - a_q,
so s_i(q) <= 2K - a_q - N_i and s_i(q) >= N_i - (a_q - 2) as well (a q near
the top has nearly all of group i below it).  The GPU filter bounds H over
these intervals; here the intervals themselves are checked against the
exactly re-ranked sums.

The kept samples' re-ranked centred values sum to zero, so the shifts obey
sum_i s_i = -(sum of the missing samples' centred ranks): the scans and the
filter bound f = sum_i D'_i^2 / N_i by its largest value over the box of
shifts cut by that plane, taken at the polygon's vertices (f is convex).
The last test checks the constraint and that this vertex maximum is never
below the exact f, for the scans' box |s_i| <= |Q| N_i and for the rank-aware
intervals.
"""
import numpy as np


def doubled_midranks(x):
    # 2 * #{j: x_j < x_k} + #{j: x_j == x_k} + 1, by brute force
    less = (x[None, :] < x[:, None]).sum(axis=1)
    eq = (x[None, :] == x[:, None]).sum(axis=1)
    return 2 * less + eq + 1


def rank_aware_interval(K, Ni, a_miss):
    """The filter's summed shift interval [lo, hi] of a group of Ni kept
    samples, from the missing samples' doubled midranks."""
    lo = -sum(min(Ni, (int(aq) - 2) // 2, int(aq) - 2 - Ni) for aq in a_miss)
    hi = sum(min(Ni, K - (int(aq) + 1) // 2, 2 * K - int(aq) - Ni) for aq in a_miss)
    return lo, hi


def test_rank_aware_interval_holds_with_ties():
    rng = np.random.default_rng(11)
    checked = tight = 0
    for _ in range(3000):
        K = int(rng.integers(3, 40))
        x = rng.integers(0, int(rng.integers(1, 8)), K).astype(float)   # many ties
        g = rng.integers(0, 3, K)
        miss = rng.random(K) < rng.uniform(0.0, 0.5)
        keep = ~miss
        if not keep.any():
            continue
        a = doubled_midranks(x)
        c = a - (K + 1)
        kp = int(keep.sum())
        cp = doubled_midranks(x[keep]) - (kp + 1)
        N = [int(((g == i) & keep).sum()) for i in range(3)]
        Dt = [int(c[(g == i) & keep].sum()) for i in range(3)]
        Dp = [int(cp[g[keep] == i].sum()) for i in range(3)]
        # group 0 from the other two and the missing samples' centred ranks
        assert Dt[0] == -Dt[1] - Dt[2] - int(c[miss].sum())
        for i in range(3):
            lo0 = -sum(min(N[i], (int(aq) - 2) // 2) for aq in a[miss])
            hi0 = sum(min(N[i], K - (int(aq) + 1) // 2) for aq in a[miss])
            lo, hi = rank_aware_interval(K, N[i], a[miss])
            assert lo0 <= lo and hi <= hi0
            tight += lo > lo0 or hi < hi0
            assert Dt[i] - hi <= Dp[i] <= Dt[i] - lo
            # one missing sample at a time: each s_i(q) inside its own interval
            for q in np.flatnonzero(miss):
                others = (g == i) & keep
                s_q = int(np.sign(x[others] - x[q]).sum())
                lq, hq = rank_aware_interval(K, N[i], [a[q]])
                assert lq <= s_q <= hq
        checked += 1
    assert checked > 2500 and tight > checked // 4


def _vertex_max(D, lo, hi, total, N):
    """Largest sum_i (D_i - s_i)^2 / N_i over lo_i <= s_i <= hi_i with
    sum_i s_i = total: two shifts at an end of their interval, the third from
    the sum and inside its own (None if no such point)."""
    best = None
    for j in range(3):
        o1, o2 = [i for i in range(3) if i != j]
        for s1 in (lo[o1], hi[o1]):
            for s2 in (lo[o2], hi[o2]):
                sj = total - s1 - s2
                if not lo[j] <= sj <= hi[j]:
                    continue
                s = [0, 0, 0]
                s[o1], s[o2], s[j] = s1, s2, sj
                f = sum((D[i] - s[i]) ** 2 / N[i] for i in range(3) if N[i])
                best = f if best is None else max(best, f)
    return best


def test_sum_constrained_bound_holds_with_ties():
    rng = np.random.default_rng(12)
    checked = tighter = 0
    for _ in range(3000):
        K = int(rng.integers(3, 40))
        x = rng.integers(0, int(rng.integers(1, 8)), K).astype(float)
        g = rng.integers(0, 3, K)
        miss = rng.random(K) < rng.uniform(0.0, 0.5)
        keep = ~miss
        if not keep.any():
            continue
        a = doubled_midranks(x)
        c = a - (K + 1)
        kp = int(keep.sum())
        cp = doubled_midranks(x[keep]) - (kp + 1)
        N = [int(((g == i) & keep).sum()) for i in range(3)]
        Dt = [int(c[(g == i) & keep].sum()) for i in range(3)]
        Dp = [int(cp[g[keep] == i].sum()) for i in range(3)]
        total = -int(c[miss].sum())
        assert sum(Dt[i] - Dp[i] for i in range(3)) == total
        exact = sum(Dp[i] ** 2 / N[i] for i in range(3) if N[i])
        nq = int(miss.sum())
        box = _vertex_max(Dt, [-nq * n for n in N], [nq * n for n in N], total, N)
        assert box is not None and box >= exact - 1e-9
        lo = [rank_aware_interval(K, N[i], a[miss])[0] for i in range(3)]
        hi = [rank_aware_interval(K, N[i], a[miss])[1] for i in range(3)]
        ranked = _vertex_max(Dt, lo, hi, total, N)
        assert ranked is not None and ranked >= exact - 1e-9
        plain = sum(max(abs(Dt[i] - hi[i]), abs(Dt[i] - lo[i])) ** 2 / N[i]
                    for i in range(3) if N[i])
        assert ranked <= plain + 1e-9
        tighter += ranked < plain - 1e-9
        checked += 1
    assert checked > 2500 and tighter > checked // 4
