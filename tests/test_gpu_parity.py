"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: ranks, tie terms, group counts and rank sums bit-exact; H equal to the
oracle's correctly rounded value (checked within 1e-12 relative, and exactly
0 where the oracle has 0); p within 1e-10 relative (absolute floor 1e-300);
hit lists identical as (trait, snp) sets in (trait, snp) order.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1307_3519_amd import datagen

pytestmark = pytest.mark.gpu

H_REL = 1e-12
P_REL = 1e-10
P_ABS = 1e-300


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kx():
    from paper_1307_3519_amd import krux
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = krux.Context(0)
    yield ctx
    ctx.close()


def _inputs(seed, T, K, M, tie_frac=0.05, p_missing=0.0, nan_frac=0.0):
    rs = datagen.streams(seed)
    x = datagen.inject_ties(rs["ties"], datagen.to_expression(
        datagen.log_normal_z(rs["expr"], T, K)), tie_frac)
    g, _ = datagen.genotypes(rs["geno"], M, K)
    g = datagen.set_missing(rs["missing"], g, p_missing)
    if nan_frac:
        mask = rs["missing"].random(x.shape) < nan_frac
        x[mask] = np.nan
    return x, g


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def assert_H(Hg, Ho, where=""):
    Hg = np.asarray(Hg); Ho = np.asarray(Ho)
    assert np.array_equal(Hg == 0, Ho == 0), where
    rel = np.abs(Hg - Ho) / np.maximum(np.abs(Ho), 1e-300)
    assert rel.max(initial=0) <= H_REL, (where, rel.max())


def assert_p(pg, po, where=""):
    pg = np.asarray(pg); po = np.asarray(po)
    bad = np.abs(pg - po) > np.maximum(P_REL * np.abs(po), P_ABS)
    assert not bad.any(), (where, pg[bad][:5], po[bad][:5])


# ---------------------------------------------------------------- rank
@pytest.mark.parametrize("K", [1, 2, 7, 48, 102, 128, 129, 500, 1000])
def test_rank_bit_exact(kx, K):
    say("rank", K)
    x, _ = _inputs(100 + K, 67, K, 1, tie_frac=0.2, nan_frac=0.02)
    x[0, : min(K, 3)] = 0.0
    if K > 3:
        x[0, 3] = -0.0
    x[1, :] = 1.5                      # all tied
    r, ts, nv = kx.rank(_dev(x))
    torch.cuda.synchronize()
    ro, tso, nvo = oracle.rank(x)
    assert np.array_equal(r.cpu().numpy().astype(np.int32), ro)
    assert np.array_equal(ts.cpu().numpy(), tso)
    assert np.array_equal(nv.cpu().numpy(), nvo)


def _ranks(kx, x):
    r, ts, nv = kx.rank(_dev(x))
    return r, ts


# ---------------------------------------------------------------- full / sums
CASES = [  # (K, T, M, p_missing)
    (5, 40, 37, 0.0), (20, 70, 100, 0.1), (33, 70, 100, 0.0), (102, 70, 161, 0.0),
    (102, 33, 65, 0.05),
    (128, 65, 64, 0.0), (48, 64, 96, 0.1), (77, 31, 40, 0.03),
    # tiled large-K kernels: ragged trait blocks (T % 128) and SNP blocks (M % 128),
    # the DIAG / PLAIN boundary at K = 400 / 401, byte-split int8 ranks
    (129, 70, 100, 0.0), (150, 140, 161, 0.0), (233, 65, 97, 0.02), (400, 40, 70, 0.0),
    (401, 36, 45, 0.0), (500, 37, 70, 0.01), (1000, 33, 40, 0.0),
    # missing genotypes at large K: re-rank scratch in the LDS ring, and at
    # the fp16 limit K = 2049 the rank bitmap no longer fits one wave (binary
    # search path)
    (1000, 40, 60, 0.02), (2049, 33, 40, 0.02)]


@pytest.mark.parametrize("prec", ["fp16", "int8", "fp64"])
@pytest.mark.parametrize("K,T,M,pm", CASES)
def test_full_and_sums(kx, prec, K, T, M, pm):
    say("full/sums", prec, K, T, M, pm)
    x, g = _inputs(7 * K + T, T, K, M, p_missing=pm)
    r, ts = _ranks(kx, x)
    gd = _dev(g)
    o = oracle.scan(x, g, full=True, sums=True)
    res = kx.test(r, ts, gd, mode="full", precision=prec)
    torch.cuda.synchronize()
    assert_H(res["H"].cpu().numpy(), o["H"], "H")
    assert_p(res["p"].cpu().numpy(), o["p"], "p")
    res = kx.test(r, ts, gd, mode="sums", precision=prec)
    torch.cuda.synchronize()
    assert np.array_equal(res["sums"].cpu().numpy().astype(np.int64), o["sums"])


# ---------------------------------------------------------------- hits
def _check_hits(kx, x, g, p_c, prec, cap=1 << 15):
    r, ts = _ranks(kx, x)
    res = kx.test(r, ts, _dev(g), p_c=p_c, mode="hits", precision=prec, hit_capacity=cap,
                  min_p=True)
    torch.cuda.synchronize()
    from paper_1307_3519_amd.krux import unpack_hits
    n, h = unpack_hits(res)
    o = oracle.scan(x, g, p_cs=(p_c,), hits=True, min_p=True)
    assert n == o["n_hits"]
    k = min(n, cap)
    if n <= cap:
        assert np.array_equal(h["trait"], o["hits"]["trait"])
        assert np.array_equal(h["snp"], o["hits"]["snp"])
        assert_H(h["H"], o["hits"]["H"], "hit H")
        assert_p(h["p"], o["hits"]["p"], "hit p")
    else:
        keys = set(zip(o["hits"]["trait"].tolist(), o["hits"]["snp"].tolist()))
        got = list(zip(h["trait"][:k].tolist(), h["snp"][:k].tolist()))
        assert got == sorted(got) and set(got) <= keys
    assert_p(res["min_p"].cpu().numpy(), o["min_p"], "min p")
    return n


@pytest.mark.parametrize("prec", ["fp16", "int8", "fp64"])
@pytest.mark.parametrize("K,T,M,pm", CASES)
def test_hits_and_min_p(kx, prec, K, T, M, pm):
    say("hits", prec, K, T, M, pm)
    x, g = _inputs(11 * K + M, T, K, M, p_missing=pm)
    n = _check_hits(kx, x, g, 0.02, prec)
    # H <= K - 1, so at K = 5 no pair reaches p < 0.02; larger K must produce hits
    assert n > 0 or K < 10


def test_hits_planted_and_capacity(kx):
    say("hits planted / capacity")
    w = datagen.make_workload(2, T=200, M=3000, n_plant=40)
    x, g = w["expr"], w["geno"]
    n = _check_hits(kx, x, g, 1e-5, "fp16")
    planted = set(map(tuple, w["planted"][:, :2].tolist()))
    assert n >= 1
    # capacity smaller than the count: true count reported, kept subset valid
    n2 = _check_hits(kx, x, g, 1e-2, "fp16", cap=7)
    assert n2 > 7
    del planted


@pytest.mark.parametrize("prec", ["fp16", "int8"])
def test_hits_many_sorted(kx, prec):
    # ~1.2e5 hits: many tiles of the hit sort, two digits of trait and SNP
    # numbers each, snp_base pushing SNP numbers past 2^16
    say("hits many", prec)
    x, g = _inputs(404, 400, 102, 6000)
    r, ts = _ranks(kx, x)
    p_c = 0.05
    res = kx.test(r, ts, _dev(g), p_c=p_c, mode="hits", precision=prec, hit_capacity=1 << 18,
                  min_p=False, snp_base=70000)
    torch.cuda.synchronize()
    from paper_1307_3519_amd.krux import unpack_hits
    n, h = unpack_hits(res)
    o = oracle.scan(x, g, p_cs=(p_c,), hits=True)
    assert n == o["n_hits"] > 100000
    assert np.array_equal(h["trait"], o["hits"]["trait"])
    assert np.array_equal(h["snp"] - 70000, o["hits"]["snp"])
    assert_H(h["H"], o["hits"]["H"], "hit H")


def test_degenerate_inputs(kx):
    say("degenerate")
    K = 40
    x, g = _inputs(5, 37, K, 50)
    x[3, :] = 2.0                      # all-tied trait: H = 0, p = 1
    g[4, :] = 1                        # monomorphic SNP: df = 0
    g[5, :20] = 0; g[5, 20:] = 2       # two groups only
    g[6, :] = -1; g[6, 7] = 1          # everything missing but one sample
    for prec in ("fp16", "int8", "fp64"):
        r, ts = _ranks(kx, x)
        res = kx.test(r, ts, _dev(g), mode="full", precision=prec)
        torch.cuda.synchronize()
        o = oracle.scan(x, g, full=True)
        assert_H(res["H"].cpu().numpy(), o["H"], prec)
        assert_p(res["p"].cpu().numpy(), o["p"], prec)
        _check_hits(kx, x, g, 0.05, prec)


def test_empty_shapes(kx):
    say("empty")
    x, g = _inputs(6, 5, 20, 0)
    r, ts = _ranks(kx, x)
    res = kx.test(r, ts, _dev(g).reshape(0, 20), p_c=0.1)
    torch.cuda.synchronize()
    assert int(res["n_hits_t"].item()) == 0
    assert np.all(res["min_p"].cpu().numpy() == 1.0)


# ---------------------------------------------------------------- permutations
@pytest.mark.parametrize("K,T,M", [(102, 70, 130), (30, 40, 64), (233, 40, 70)])
def test_permute_counts_and_min_p(kx, K, T, M):
    say("permute", K, T, M)
    x, g = _inputs(13 + K, T, K, M)
    rs = datagen.streams(99)
    perms = datagen.permutations(rs["perms"], 5, K)
    r, ts = _ranks(kx, x)
    p_cs = (0.05, 0.01, 0.001)
    res = kx.permute(r, ts, _dev(g), _dev(perms), p_cs=p_cs)
    torch.cuda.synchronize()
    counts = res["counts"].cpu().numpy()
    mp = res["min_p"].cpu().numpy()
    for i in range(perms.shape[0]):
        o = oracle.scan(x, g, p_cs=p_cs, perm=perms[i], min_p=True)
        assert np.array_equal(counts[i], o["counts"]), i
        assert_p(mp[i], o["min_p"], "perm min p")


def test_permute_large_operand(kx):
    # 50 permutations x 1500 traits: a 16 MB operand, screened through the
    # block-shared LDS ring pipeline
    K, T, M, P = 102, 1500, 97, 50
    say("permute large operand", K, T, M, P)
    x, g = _inputs(29, T, K, M)
    rs = datagen.streams(31)
    perms = datagen.permutations(rs["perms"], P, K)
    r, ts = _ranks(kx, x)
    p_cs = (0.05, 0.01, 0.001)
    res = kx.permute(r, ts, _dev(g), _dev(perms), p_cs=p_cs)
    torch.cuda.synchronize()
    counts = res["counts"].cpu().numpy()
    mp = res["min_p"].cpu().numpy()
    for i in range(P):
        o = oracle.scan(x, g, p_cs=p_cs, perm=perms[i], min_p=True)
        assert np.array_equal(counts[i], o["counts"]), i
        assert_p(mp[i], o["min_p"], "perm min p %d" % i)


# ---------------------------------------------------------------- small workload, full size
def test_small_workload_full_matrices(kx):
    say("workload small_full 1000 x 2000 x 102")
    w = datagen.make_workload(1)
    x, g = w["expr"], w["geno"]
    r, ts = _ranks(kx, x)
    res = kx.test(r, ts, _dev(g), mode="full", precision="fp16")
    torch.cuda.synchronize()
    o = oracle.scan(x, g, full=True)
    assert_H(res["H"].cpu().numpy(), o["H"], "H")
    assert_p(res["p"].cpu().numpy(), o["p"], "p")
    assert np.array_equal(res["H"].cpu().numpy(), o["H"])   # correctly rounded on both sides


def test_heavy_missing_per_snp(kx):
    # SNPs with 0 .. 200 missing samples: listed positions (up to 32) and the
    # packed-row bound beyond, the sorted-rank re-rank (up to 64 missing) and
    # the pairwise one (more than 64), ties in every trait
    say("heavy missing")
    K, T, M = 233, 50, 48
    x, g = _inputs(61, T, K, M, tie_frac=0.2)
    rs = datagen.streams(62)["missing"]
    for m, nmiss in enumerate([0, 1, 5, 30, 32, 33, 63, 64, 65, 100, 150, 200] * 4):
        idx = rs.choice(K, size=nmiss, replace=False)
        g[m, idx] = -1
    r, ts = _ranks(kx, x)
    o = oracle.scan(x, g, full=True, p_cs=(0.05,), hits=True, min_p=True)
    for prec in ("fp16", "int8"):
        res = kx.test(r, ts, _dev(g), mode="full", precision=prec)
        torch.cuda.synchronize()
        assert_H(res["H"].cpu().numpy(), o["H"], prec)
        assert_p(res["p"].cpu().numpy(), o["p"], prec)
        _check_hits(kx, x, g, 0.05, prec)


# ------------------------------------------------- missing expression values
# Traits with NaN entries (rank 0): each pair keeps the samples with both an
# expression value and a genotype (K' per pair, group sizes per pair), with
# and without missing genotypes; the SNP-stationary (K <= 128) and tiled
# kernels, every precision and mode.
NAN_CASES = [(48, 40, 70, 0.0), (102, 37, 65, 0.03), (233, 36, 70, 0.02)]


@pytest.mark.parametrize("prec", ["fp16", "int8", "fp64"])
@pytest.mark.parametrize("K,T,M,pm", NAN_CASES)
def test_missing_expression(kx, prec, K, T, M, pm):
    say("nan", prec, K, T, M, pm)
    x, g = _inputs(17 * K + T, T, K, M, p_missing=pm, nan_frac=0.03)
    x[2, :] = np.nan                   # no expression value at all: H = 0, p = 1
    x[3, 1:] = np.nan                  # a single one
    assert np.isnan(x).any(axis=1).sum() > T // 3
    r, ts = _ranks(kx, x)
    gd = _dev(g)
    o = oracle.scan(x, g, full=True, sums=True)
    res = kx.test(r, ts, gd, mode="full", precision=prec)
    torch.cuda.synchronize()
    assert_H(res["H"].cpu().numpy(), o["H"], "H")
    assert_p(res["p"].cpu().numpy(), o["p"], "p")
    res = kx.test(r, ts, gd, mode="sums", precision=prec)
    torch.cuda.synchronize()
    assert np.array_equal(res["sums"].cpu().numpy().astype(np.int64), o["sums"])
    _check_hits(kx, x, g, 0.02, prec)


def test_permute_missing_expression(kx):
    say("permute nan")
    K, T, M = 48, 30, 50
    x, g = _inputs(29, T, K, M, p_missing=0.02, nan_frac=0.05)
    rs = datagen.streams(98)
    perms = datagen.permutations(rs["perms"], 4, K)
    r, ts = _ranks(kx, x)
    p_cs = (0.05, 0.01)
    res = kx.permute(r, ts, _dev(g), _dev(perms), p_cs=p_cs)
    torch.cuda.synchronize()
    counts = res["counts"].cpu().numpy()
    mp = res["min_p"].cpu().numpy()
    for i in range(perms.shape[0]):
        o = oracle.scan(x, g, p_cs=p_cs, perm=perms[i], min_p=True)
        assert np.array_equal(counts[i], o["counts"]), i
        assert_p(mp[i], o["min_p"], "perm min p")


# ---------------------------------------------------------------- empirical FDR curve
FDR_CASES = [  # (K, T, M, p_missing, nan_frac, P)
    (48, 30, 120, 0.0, 0.0, 5),
    (102, 37, 90, 0.02, 0.02, 4),
    (233, 20, 70, 0.02, 0.0, 3),
]


@pytest.mark.parametrize("K,T,M,pm,nan,P", FDR_CASES)
def test_permute_hits_and_fdr_curve(kx, K, T, M, pm, nan, P):
    from paper_1307_3519_amd.krux import unpack_hits
    say("fdr", K, T, M, pm, nan, P)
    x, g = _inputs(31 * K + T, T, K, M, p_missing=pm, nan_frac=nan)
    perms = datagen.permutations(datagen.streams(K + 7)["perms"], P, K)
    r, ts = _ranks(kx, x)
    gd, pd = _dev(g), _dev(perms)
    p_c = 0.02
    ph = kx.permute_hits(r, ts, gd, pd, p_c=p_c, hit_capacity=1 << 14)
    real = kx.test(r, ts, gd, p_c=p_c, mode="hits", precision="fp16", hit_capacity=1 << 14,
                   min_p=False)
    fdr = kx.fdr_curve(real, ph, P)
    torch.cuda.synchronize()
    n_p, hp = unpack_hits(ph)
    n_r, hr = unpack_hits(real)
    # the permuted hits, permutation by permutation (rows perm * T + trait)
    o_perm_p, tot = [], 0
    for i in range(P):
        o = oracle.scan(x, g, p_cs=(p_c,), perm=perms[i], hits=True)
        sel = (hp["trait"] // T) == i
        assert np.array_equal(hp["trait"][sel] % T, o["hits"]["trait"]), i
        assert np.array_equal(hp["snp"][sel], o["hits"]["snp"]), i
        assert_p(hp["p"][sel], o["hits"]["p"], "permuted hit p")
        o_perm_p.append(o["hits"]["p"])
        tot += o["n_hits"]
    assert n_p == tot and n_p > 0 and n_r > 0
    f = fdr[:n_r].cpu().numpy()
    # the curve from the GPU's own p-values, exactly as the definition counts
    assert np.array_equal(f, oracle.fdr_curve(hr["p"], hp["p"], P))
    # and from the oracle's hit lists
    o_real = oracle.scan(x, g, p_cs=(p_c,), hits=True)
    assert np.array_equal(f, oracle.fdr_curve(o_real["hits"]["p"], np.concatenate(o_perm_p), P))
    # no permuted hit: FDR 0 at every real hit
    ph0 = kx.permute_hits(r, ts, gd, pd, p_c=1e-300, hit_capacity=16)
    f0 = kx.fdr_curve(real, ph0, P)
    torch.cuda.synchronize()
    assert unpack_hits(ph0)[0] == 0 and np.all(f0[:n_r].cpu().numpy() == 0.0)
    # capacity below the count: the true count, a valid subset kept
    small = kx.permute_hits(r, ts, gd, pd, p_c=p_c, hit_capacity=3)
    torch.cuda.synchronize()
    n_s, hs = unpack_hits(small)
    assert n_s == tot and len(hs["snp"]) == 3
    full = set(zip(hp["trait"].tolist(), hp["snp"].tolist()))
    assert set(zip(hs["trait"].tolist(), hs["snp"].tolist())) <= full


def test_missing_expression_heavy_ties(kx):
    # few distinct values: removed samples often share a tie group, the
    # tie-term update then depends on the order of removals
    say("nan heavy ties")
    K, T, M = 40, 30, 90
    x, g = _inputs(77, T, K, M, p_missing=0.06, nan_frac=0.05)
    x = np.where(np.isnan(x), x, np.round(x * 2.0) / 2.0).astype(np.float32)
    r, ts = _ranks(kx, x)
    gd = _dev(g)
    o = oracle.scan(x, g, full=True, sums=True)
    res = kx.test(r, ts, gd, mode="full", precision="fp16")
    torch.cuda.synchronize()
    assert_H(res["H"].cpu().numpy(), o["H"], "H")
    assert_p(res["p"].cpu().numpy(), o["p"], "p")
    res = kx.test(r, ts, gd, mode="sums", precision="fp16")
    torch.cuda.synchronize()
    assert np.array_equal(res["sums"].cpu().numpy().astype(np.int64), o["sums"])
    _check_hits(kx, x, g, 0.05, "fp16")


# ---------------------------------------------------------------- missing-pattern groups
GROUP_CASES = [  # (K, T, M, precision)
    (102, 40, 600, "fp16"),
    (48, 30, 400, "int8"),
    (233, 25, 300, "fp16"),
    (102, 20, 300, "fp64"),
]


@pytest.mark.parametrize("K,T,M,prec", GROUP_CASES)
def test_grouped_patterns(kx, K, T, M, prec):
    from paper_1307_3519_amd.krux import unpack_hits
    say("grouped", K, T, M, prec)
    x, g = _inputs(41 * K + T, T, K, M, nan_frac=0.02)
    rs = datagen.streams(K + T)
    g = datagen.set_missing_samples(rs["missing"], g, [[3, 17, K - 1], [8]], [0.6, 0.2])
    g = datagen.set_missing(rs["cohort"], g, 0.003)       # sporadic: patterns of their own
    r, ts = _ranks(kx, x)
    gd = _dev(g)
    p_c = 0.02
    res = kx.test_grouped(r, ts, gd, p_c=p_c, precision=prec, min_group=16,
                          hit_capacity=1 << 15, snp_base=5)
    ref = kx.test(r, ts, gd, p_c=p_c, mode="hits", precision=prec, hit_capacity=1 << 15,
                  min_p=True, snp_base=5)
    torch.cuda.synchronize()
    o = oracle.scan(x, g, p_cs=(p_c,), hits=True, min_p=True)
    n, h = unpack_hits(res)
    assert n == o["n_hits"] and n > 0
    assert np.array_equal(h["trait"], o["hits"]["trait"])
    assert np.array_equal(h["snp"] - 5, o["hits"]["snp"])
    assert_H(h["H"], o["hits"]["H"], "grouped H")
    assert_p(h["p"], o["hits"]["p"], "grouped p")
    assert_p(res["min_p"].cpu().numpy(), o["min_p"], "grouped min p")
    # the same bits as the ungrouped scan
    n2, h2 = unpack_hits(ref)
    assert n2 == n
    for f in ("trait", "snp", "H", "p"):
        assert np.array_equal(h[f], h2[f]), f
    assert np.array_equal(res["min_p"].cpu().numpy(), ref["min_p"].cpu().numpy())
    # capacity below the count: the true count and a valid subset
    small = kx.test_grouped(r, ts, gd, p_c=p_c, precision=prec, min_group=16, hit_capacity=4)
    torch.cuda.synchronize()
    n_s, hs = unpack_hits(small)
    assert n_s == n and len(hs["snp"]) == 4
    assert set(zip(hs["trait"].tolist(), hs["snp"].tolist())) <= \
        set(zip(h["trait"].tolist(), (h["snp"] - 5).tolist()))


def test_new_entry_points_reject_bad_arguments(kx):
    from paper_1307_3519_amd import krux
    say("argument errors")
    x, g = _inputs(5, 8, 20, 30)
    r, ts = _ranks(kx, x)
    gd = _dev(g)
    perms = _dev(datagen.permutations(datagen.streams(5)["perms"], 2, 20))
    with pytest.raises(krux.KruxError):
        kx.test_grouped(r, ts, gd, min_group=0)
    with pytest.raises(krux.KruxError):
        kx.test_grouped(r, ts, gd, p_c=0.0)
    with pytest.raises(krux.KruxError):
        kx.permute_hits(r, ts, gd, perms, p_c=1.5)
    for G in (1, 9):
        with pytest.raises(krux.KruxError):
            kx.test_multi(r, ts, gd, G)
    with pytest.raises(krux.KruxError):
        kx.test_multi(r, ts, gd, 4, mode="sums")
    real = kx.test(r, ts, gd, p_c=0.5, mode="hits", hit_capacity=64)
    ph = kx.permute_hits(r, ts, gd, perms, p_c=0.5, hit_capacity=64)
    with pytest.raises(krux.KruxError):
        kx.fdr_curve(real, ph, 0)
    torch.cuda.synchronize()
    # the context still works after the rejected calls
    f = kx.fdr_curve(real, ph, 2)
    torch.cuda.synchronize()
    n = int(real["n_hits_t"].item())
    assert n > 0 and np.all(np.isfinite(f[:n].cpu().numpy()))


def test_grouped_degenerate_cases(kx):
    # no pattern reaches min_group, complete genotypes, a pattern that removes
    # every sample but one, and an empty SNP panel: all equal krux_test
    from paper_1307_3519_amd.krux import unpack_hits
    say("grouped degenerate")
    K, T, M = 30, 12, 120
    x, g = _inputs(9, T, K, M)
    g_one = g.copy()
    g_one[:60, 1:] = -1                    # 60 SNPs keep only sample 0
    for gg, mg in ((g, 4), (datagen.set_missing(datagen.streams(3)["missing"], g, 0.05), 1000),
                   (g_one, 8), (g[:0], 1)):
        r, ts = _ranks(kx, x)
        gd = _dev(gg)
        res = kx.test_grouped(r, ts, gd, p_c=0.05, min_group=mg, hit_capacity=4096)
        ref = kx.test(r, ts, gd, p_c=0.05, mode="hits", hit_capacity=4096, min_p=True)
        torch.cuda.synchronize()
        a, b = unpack_hits(res), unpack_hits(ref)
        assert a[0] == b[0]
        for f in ("trait", "snp", "H", "p"):
            assert np.array_equal(a[1][f], b[1][f]), f
        assert np.array_equal(res["min_p"].cpu().numpy(), ref["min_p"].cpu().numpy())


# ---------------------------------------------------------------- multi-allelic markers
# (K, T, M, n_classes, missing genotypes, NaN values): the MFMA screen takes
# the complete pairs at K <= 128 with up to five classes (one to eight
# k-steps, one to four indicator columns), the lane kernel every other pair
MULTI_CASES = [
    (40, 8, 70, 4, 0.03, 0.03),
    (37, 6, 65, 6, 0.03, 0.03),
    (150, 5, 30, 5, 0.03, 0.03),
    (30, 5, 40, 8, 0.03, 0.03),
    (102, 40, 130, 4, 0.0, 0.0),
    (102, 37, 100, 4, 0.005, 0.005),
    (17, 35, 70, 3, 0.0, 0.0),
    (128, 33, 64, 5, 0.0, 0.0),
    (64, 40, 90, 2, 0.0, 0.0),
    (90, 36, 80, 5, 0.0, 0.0),
    (1000, 3, 5, 4, 0.02, 0.0),
    (700, 3, 6, 8, 0.02, 0.02),
]


def _multi_inputs(K, T, M, G, pm, nan):
    rng = np.random.default_rng(K * 100 + G + T)
    x = np.round(rng.lognormal(size=(T, K)), 1).astype(np.float32)      # ties
    if nan:
        x[rng.random(x.shape) < nan] = np.nan
        x[0, :] = np.nan
    q = rng.dirichlet(np.ones(G), size=M)
    g = np.array([rng.choice(G, size=K, p=q[m]) for m in range(M)], dtype=np.int8)
    if pm:
        g[rng.random(g.shape) < pm] = -1
        g[rng.random(g.shape) < pm / 3] = G + 1                          # also missing
    g[1, :] = 0                                                          # one class only
    # an effect on a few traits so that small p-values occur
    for t in range(2, min(T, 6)):
        m = 2 + t
        x[t] = np.where(np.isnan(x[t]), x[t], x[t] + 0.7 * np.clip(g[m], 0, G)).astype(np.float32)
    return x, g


@pytest.mark.parametrize("K,T,M,G,pm,nan", MULTI_CASES)
def test_multi_allelic(kx, K, T, M, G, pm, nan):
    from oracle import multi
    from paper_1307_3519_amd.krux import unpack_hits
    say("multi", K, T, M, G, pm, nan)
    x, g = _multi_inputs(K, T, M, G, pm, nan)
    r, ts = _ranks(kx, x)
    gd = _dev(g)
    p_c = 0.05
    o = multi.scan(x, g, G, p_c=p_c)
    full = kx.test_multi(r, ts, gd, G, mode="full")
    res = kx.test_multi(r, ts, gd, G, p_c=p_c, mode="hits", hit_capacity=1 << 14, snp_base=3)
    torch.cuda.synchronize()
    # H is the correctly rounded rational on both sides
    assert np.array_equal(full["H"].cpu().numpy(), o["H"])
    assert_p(full["p"].cpu().numpy(), o["p"], "multi p")
    n, h = unpack_hits(res)
    assert n == len(o["hits"]) and n > 0
    assert list(zip(h["trait"].tolist(), (h["snp"] - 3).tolist())) == o["hits"]
    assert np.array_equal(h["H"], o["H"][h["trait"], h["snp"] - 3])
    assert_p(res["min_p"].cpu().numpy(), o["p"].min(axis=1), "multi min p")


def test_multi_allelic_small_p_and_overflow():
    # the MFMA screen at p < 1e-4 (few candidates) and with a candidate
    # buffer of 8 entries (the rest evaluated inside the screen kernel)
    from oracle import multi
    from paper_1307_3519_amd import krux
    from paper_1307_3519_amd.krux import unpack_hits
    say("multi small p / overflow")
    K, T, M, G = 102, 40, 120, 4
    x, g = _multi_inputs(K, T, M, G, 0.0, 0.0)
    o = multi.scan(x, g, G)
    for limit, p_c in ((0, 1e-4), (8, 0.05)):
        ctx = krux.Context(0)
        try:
            ctx.set_pair_buffer_limits(limit, 0)
            r, ts, _ = ctx.rank(_dev(x))
            res = ctx.test_multi(r, ts, _dev(g), G, p_c=p_c, mode="hits", hit_capacity=1 << 14)
            torch.cuda.synchronize()
            n, h = unpack_hits(res)
            want = [(t, m) for t in range(T) for m in range(M)
                    if o["p"][t, m] < 1.0 and o["H"][t, m] > multi.threshold(
                        p_c, multi.one_pair(x[t], g[m], G)["df"])]
            assert n == len(want) and list(zip(h["trait"].tolist(), h["snp"].tolist())) == want
            assert_p(res["min_p"].cpu().numpy(), o["p"].min(axis=1), "multi min p")
        finally:
            ctx.close()
