"""The bound behind the re-rank filter for SNPs with missing genotypes
(sample exclusion with re-ranking over the rest, section 2), checked by
brute force on small inputs with heavy ties.

Removing missing sample q shifts the centred rank sum of group i by
-s_i(q), s_i(q) = #{kept k in group i above q} - #{kept k in group i below q};
from q's doubled midrank a_q alone, at most (a_q - 2) / 2 samples lie below q
and at most K - a_q / 2 above it, so s_i(q) lies in
[-min(N_i, (a_q - 2) // 2), min(N_i, K - (a_q + 1) // 2)].  The GPU filter
bounds H over these intervals; here the intervals themselves are checked
against the exactly re-ranked sums.
"""
import numpy as np


def doubled_midranks(x):
    # 2 * #{j: x_j < x_k} + #{j: x_j == x_k} + 1, by brute force
    less = (x[None, :] < x[:, None]).sum(axis=1)
    eq = (x[None, :] == x[:, None]).sum(axis=1)
    return 2 * less + eq + 1


def test_rank_aware_interval_holds_with_ties():
    rng = np.random.default_rng(11)
    checked = 0
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
            lo = -sum(min(N[i], (int(aq) - 2) // 2) for aq in a[miss])
            hi = sum(min(N[i], K - (int(aq) + 1) // 2) for aq in a[miss])
            assert Dt[i] - hi <= Dp[i] <= Dt[i] - lo
        checked += 1
    assert checked > 2500
