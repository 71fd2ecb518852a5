"""Pins for the multi-allelic oracle (oracle/multi.py): facts fixed by the
mathematics, independent of its code.

  scipy        scipy.stats.kruskal with 4-6 groups; scipy.stats.chi2.sf
  C oracle     two alleles (classes 0..2): the same H as the C oracle
  brute force  the exact permutation-null mean E[H] = df for 4 groups
  threshold    the largest double with p >= p_c; the C oracle's for df 1, 2
"""
import itertools
import math

import numpy as np
import pytest
import scipy.stats as st

import oracle
from oracle import multi
from paper_1307_3519_amd import datagen


def test_chi2_tail_matches_scipy():
    for df in range(1, 9):
        for H in (0.0, 1e-6, 0.3, 1.0, 2.5, 7.0, 15.0, 40.0, 90.0, 200.0):
            want = st.chi2.sf(H, df)
            got = multi.chi2_tail(H, df)
            assert got == pytest.approx(want, rel=1e-12, abs=1e-300), (df, H)


def test_threshold_is_largest_double_with_p_at_least_pc():
    for df in (1, 2, 3, 4, 5, 7):
        for pc in (0.5, 1e-3, 1e-5, 1e-8):
            h = multi.threshold(pc, df)
            assert multi.chi2_tail(h, df) >= pc
            assert multi.chi2_tail(math.nextafter(h, math.inf), df) < pc
    for df in (1, 2):
        for pc in (0.3, 1e-4, 1e-6):
            assert multi.threshold(pc, df) == pytest.approx(oracle.threshold(pc, df), rel=1e-15)


def test_two_alleles_equal_the_c_oracle():
    rs = datagen.streams(23)
    K = 45
    x = datagen.inject_ties(rs["ties"], datagen.to_expression(
        datagen.log_normal_z(rs["expr"], 25, K)), 0.1)
    g, _ = datagen.genotypes(rs["geno"], 25, K)
    g = datagen.set_missing(rs["missing"], g, 0.05)
    x[rs["missing"].random(x.shape) < 0.03] = np.nan
    for t in range(25):
        o = oracle.one_pair(x[t], g[t])
        m = multi.one_pair(x[t], g[t], 3)
        assert m["H"] == o["H"] and m["df"] == o["df"] and m["tiesum"] == o["tiesum"]
        assert list(m["s2"]) == list(o["s2"])
        assert m["p"] == pytest.approx(o["p"], rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("G", [4, 5, 6])
def test_vs_scipy_kruskal(G):
    rng = np.random.default_rng(G)
    K = 60
    for _ in range(20):
        x = np.round(rng.lognormal(size=K), 1).astype(np.float32)     # ties
        g = rng.integers(0, G, size=K)
        g[rng.random(K) < 0.05] = G + 2                               # missing codes
        x[rng.random(K) < 0.03] = np.nan
        keep = (~np.isnan(x)) & (g < G)
        groups = [x[keep & (g == c)].astype(np.float64) for c in range(G)]
        groups = [q for q in groups if len(q)]
        o = multi.one_pair(x, g, G)
        assert o["df"] == len(groups) - 1
        r = st.kruskal(*groups)
        assert o["H"] == pytest.approx(r.statistic, rel=1e-10)
        assert o["p"] == pytest.approx(r.pvalue, rel=1e-9, abs=1e-300)


def test_permutation_null_mean_is_df():
    # 7 distinct values in 4 groups of sizes (2, 2, 2, 1): over all 630
    # assignments of samples to groups, the mean of H is exactly df = 3
    x = np.array([0.3, 1.1, 2.0, 2.7, 3.5, 4.2, 5.9], np.float32)
    labels = [0, 0, 1, 1, 2, 2, 3]
    Hs = set()
    total, count = 0.0, 0
    for perm in set(itertools.permutations(labels)):
        o = multi.one_pair(x, np.array(perm), 4)
        total += o["H"]
        count += 1
        Hs.add(o["H"])
    assert count == 630 and len(Hs) > 10
    assert total / count == pytest.approx(3.0, rel=1e-12)


def test_perfect_separation_closed_form():
    # G groups of n samples each, ordered: H = 3(K-1)/(K^3-K) * sum D_c^2/n
    # with D_c = n (2 c n + n + 1) - n (K + 1) in doubled ranks
    for G, n in ((4, 3), (5, 2), (6, 4)):
        K = G * n
        x = np.arange(K, dtype=np.float32)
        g = np.repeat(np.arange(G), n)
        o = multi.one_pair(x, g, G)
        D = [n * (2 * c * n + n + 1) - n * (K + 1) for c in range(G)]
        want = 3 * (K - 1) * sum(d * d / n for d in D) / (K ** 3 - K)
        assert o["H"] == pytest.approx(want, rel=1e-14)
        assert o["df"] == G - 1


def _scan_case(seed, T=6, M=40, K=36, G=5):
    rng = np.random.default_rng(seed)
    x = np.round(rng.lognormal(size=(T, K)), 1).astype(np.float32)      # ties
    x[rng.random(x.shape) < 0.03] = np.nan
    q = rng.dirichlet(np.ones(G), size=M)
    g = np.array([rng.choice(G, size=K, p=q[m]) for m in range(M)], dtype=np.int8)
    g[rng.random(g.shape) < 0.04] = -1
    # strong effects on a few pairs so that both sides of the threshold occur
    for t in range(T):
        m = int(rng.integers(0, M))
        x[t] = np.where(np.isnan(x[t]), x[t], x[t] + 0.8 * g[m].clip(0)).astype(np.float32)
    return x, g


def test_scan_hits_follow_scipy_tail_below_pc():
    # Hit rule (P-value calculation, strict reading): a pair is a hit iff its
    # degrees of freedom are at least 1 and its chi-square p-value is below
    # P_c.  Checked pair by pair against scipy: H from kruskal over the kept
    # samples, df from the number of classes present, p from chi2.sf; pairs
    # whose p lies within 1e-9 (relative) of P_c are left out, where the two
    # tails may round differently.
    G, p_c = 5, 0.01
    x, g = _scan_case(3, G=G)
    o = multi.scan(x, g, G, p_c=p_c)
    hits = set(o["hits"])
    assert o["hits"] == sorted(o["hits"])
    n_hit = n_miss = 0
    for t in range(x.shape[0]):
        for m in range(g.shape[0]):
            keep = (~np.isnan(x[t])) & (g[m] >= 0) & (g[m] < G)
            groups = [x[t][keep & (g[m] == c)].astype(np.float64) for c in range(G)]
            groups = [q for q in groups if len(q)]
            df = len(groups) - 1
            if df < 1 or len(np.unique(np.concatenate(groups))) < 2:
                assert (t, m) not in hits
                continue
            pv = st.chi2.sf(st.kruskal(*groups).statistic, df)
            if abs(pv - p_c) <= 1e-9 * p_c:
                continue
            want = pv < p_c
            assert ((t, m) in hits) == want, (t, m, pv, df)
            n_hit += want
            n_miss += not want
    assert n_hit >= 3 and n_miss >= 3


def test_scan_pair_at_exactly_pc_is_not_a_hit():
    # A pair whose p-value equals P_c is not a hit (strict p < P_c); with
    # P_c one ulp above its p it is.  The pair is chosen where the tail
    # falls from one double of H to the next, so that P_c = p(H) pins the
    # threshold to H itself.
    G = 5
    x, g = _scan_case(4, T=4, M=25, G=G)
    o = multi.scan(x, g, G)
    chosen = None
    for t in range(x.shape[0]):
        for m in range(g.shape[0]):
            H = o["H"][t, m]
            one = multi.one_pair(x[t], g[m], G)
            if one["df"] >= 2 and H > 1.0:
                pc = multi.chi2_tail(H, one["df"])
                if multi.chi2_tail(math.nextafter(H, math.inf), one["df"]) < pc and pc > 1e-12:
                    chosen = (t, m, pc)
                    break
        if chosen:
            break
    assert chosen is not None
    t, m, pc = chosen
    assert (t, m) not in multi.scan(x, g, G, p_c=pc)["hits"]
    assert (t, m) in multi.scan(x, g, G, p_c=math.nextafter(pc, 1.0))["hits"]


# Planted mistakes in the multi-allelic oracle must each fail one of the pins
# above (the source is edited in memory and loaded as a separate module).
MULTI_MUTATIONS = {
    "drop_tie_term": ("E = kp ** 3 - kp - tiesum", "E = kp ** 3 - kp"),
    "wrong_centre": ("(s2[c] - n[c] * (kp + 1)) ** 2", "(s2[c] - n[c] * kp) ** 2"),
    "df_off_by_one": ("df = nonempty - 1 if nonempty > 0 else 0", "df = nonempty if nonempty > 0 else 0"),
    "odd_tail_no_erfc": ("total = math.erfc(math.sqrt(x))", "total = 0.0"),
    "even_tail_sum_short": ("for k in range(1, df // 2):", "for k in range(1, df // 2 - 1):"),
    "missing_code_kept": ("(g >= 0) & (g < n_classes)", "(g < n_classes)"),
    "rank_ties_not_averaged": ("2 * less + eq + 1", "2 * less + 1"),
    "scan_hit_at_threshold": ('o["H"] > threshold(p_c, o["df"])', 'o["H"] >= threshold(p_c, o["df"])'),
    "scan_df_plus_one": ('threshold(p_c, o["df"])', 'threshold(p_c, o["df"] + 1)'),
    "scan_df_minus_one": ('threshold(p_c, o["df"])', 'threshold(p_c, max(o["df"] - 1, 1))'),
}

MULTI_BATTERY = ["test_chi2_tail_matches_scipy", "test_threshold_is_largest_double_with_p_at_least_pc",
                 "test_two_alleles_equal_the_c_oracle", "test_vs_scipy_kruskal",
                 "test_permutation_null_mean_is_df", "test_perfect_separation_closed_form",
                 "test_scan_hits_follow_scipy_tail_below_pc",
                 "test_scan_pair_at_exactly_pc_is_not_a_hit"]


@pytest.mark.parametrize("name", sorted(MULTI_MUTATIONS))
def test_planted_multi_mistake_is_caught(name, monkeypatch):
    import types
    old, new = MULTI_MUTATIONS[name]
    src = open(multi.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("multi_mutant")
    exec(compile(src.replace(old, new), "multi_mutant", "exec"), mod.__dict__)
    monkeypatch.setattr(__import__("oracle").multi, "chi2_tail", mod.chi2_tail)
    monkeypatch.setattr(__import__("oracle").multi, "threshold", mod.threshold)
    monkeypatch.setattr(__import__("oracle").multi, "one_pair", mod.one_pair)
    monkeypatch.setattr(__import__("oracle").multi, "scan", mod.scan)
    caught = []
    for t in MULTI_BATTERY:
        fn = globals()[t]
        try:
            if t == "test_vs_scipy_kruskal":
                for G in (4, 5, 6):
                    fn(G)
            else:
                fn()
        except (AssertionError, ValueError, ZeroDivisionError, OverflowError, IndexError):
            caught.append(t)
    assert caught, "mutation %s passed every pin" % name
