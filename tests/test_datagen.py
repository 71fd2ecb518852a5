"""The synthetic inputs have the shapes and structure stated for each workload."""
import numpy as np

from paper_1307_3519_amd import datagen


def test_small_workload_structure():
    w = datagen.make_workload(1)
    x, g = w["expr"], w["geno"]
    assert x.shape == (1000, 102) and x.dtype == np.float32
    assert g.shape == (2000, 102) and g.dtype == np.int8
    assert set(np.unique(g)) <= {0, 1, 2}
    # ~10% of SNPs miss one genotype class at K=102 (df = 1)
    present = np.stack([(g == c).any(axis=1) for c in range(3)], 1).sum(1)
    assert 0.075 <= np.mean(present == 2) <= 0.11
    # ties: every row has repeated values
    n_unique = np.array([len(np.unique(r)) for r in x])
    assert np.all(n_unique <= 102 - 1) and np.mean(n_unique) >= 102 - 5.5
    # determinism
    w2 = datagen.make_workload(1)
    assert np.array_equal(w2["expr"], x) and np.array_equal(w2["geno"], g)


def test_planted_and_missing_and_perms():
    w = datagen.make_workload(2, T=300, M=4000, n_plant=50)
    assert w["planted"].shape == (50, 3)
    assert len(np.unique(w["planted"][:, 0])) == 50
    for t, m, _ in w["planted"]:
        assert min((w["geno"][m] == c).sum() for c in range(3)) >= 2
    w = datagen.make_workload(4, T=10, M=10, P=7)
    assert w["perms"].shape == (7, 102)
    for p in w["perms"]:
        assert np.array_equal(np.sort(p), np.arange(102))
    cs = datagen.make_cohorts(M=500, T_scale=0.01)
    assert [c["K"] for c in cs] == list(datagen.COHORT_K)
    frac = np.mean(np.concatenate([(c["geno"] == -1).ravel() for c in cs]))
    assert 0.015 < frac < 0.025


def test_nan_expression_recipe():
    x = np.ones((4000, 102), np.float32)
    y = datagen.set_nan_expression(datagen.streams(5)["nan"], x, 0.02, 5)
    assert not np.isnan(x).any()                       # input untouched
    per = np.isnan(y).sum(axis=1)
    rows = per > 0
    assert 40 <= rows.sum() <= 130                      # about 2 % of 4000
    assert per[rows].min() >= 1 and per.max() <= 5
    assert np.array_equal(y[~np.isnan(y)], x[~np.isnan(y)])
    # the other streams do not move when the NaN stream is drawn from
    a = datagen.streams(5)["expr"].random(3)
    rs = datagen.streams(5)
    datagen.set_nan_expression(rs["nan"], x, 0.5, 3)
    assert np.array_equal(a, rs["expr"].random(3))


def test_sample_structured_missing():
    g = np.zeros((2000, 50), np.int8)
    out = datagen.set_missing_samples(datagen.streams(6)["missing"], g, [[1, 7, 49], [3]],
                                      [0.5, 0.25])
    assert not (g < 0).any()
    miss = out < 0
    a = miss[:, [1, 7, 49]].all(axis=1)
    assert np.array_equal(a, miss[:, [1, 7, 49]].any(axis=1))     # all or none
    assert 850 <= a.sum() <= 1150
    assert 380 <= miss[:, 3].sum() <= 620
    assert miss.sum() == 3 * a.sum() + miss[:, 3].sum()
