"""GPU parity of paths that the default buffer sizes rarely reach, and of the
batched-cohort entry point.

  overflow   with krux_set_pair_buffer_limits set to a few entries, the
             screened pairs that do not fit the candidate buffer are
             evaluated inside the scan kernels (eval_candidate_fallback), and
             pairs of SNPs with missing genotypes that do not fit their buffer
             are re-ranked inside the scan kernels (the in-scan drain); hits,
             per-trait minimum p and permutation counts must still equal the
             oracle's
  batched    krux_test_batched over the eight cohort sample counts of the
             uneven-cohort workload, 2% missing genotypes, each cohort's hit
             list and minimum p against the oracle
  capture    a call that would have to grow a scratch buffer while its stream
             is being captured is refused; a larger call after a capture gets
             new buffers and the captured graph still replays correctly
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1307_3519_amd import datagen

pytestmark = pytest.mark.gpu

P_REL = 1e-10
P_ABS = 1e-300
H_REL = 1e-12


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _inputs(seed, T, K, M, p_missing=0.0, nan_frac=0.0):
    rs = datagen.streams(seed)
    x = datagen.inject_ties(rs["ties"], datagen.to_expression(
        datagen.log_normal_z(rs["expr"], T, K)), 0.05)
    g, _ = datagen.genotypes(rs["geno"], M, K)
    g = datagen.set_missing(rs["missing"], g, p_missing)
    if nan_frac:
        x[rs["nan"].random(x.shape) < nan_frac] = np.nan
    return x, g


def assert_p(pg, po, where=""):
    pg = np.asarray(pg); po = np.asarray(po)
    bad = np.abs(pg - po) > np.maximum(P_REL * np.abs(po), P_ABS)
    assert not bad.any(), (where, pg[bad][:5], po[bad][:5])


def assert_hits(res, o, where=""):
    from paper_1307_3519_amd.krux import unpack_hits
    n, h = unpack_hits(res)
    assert n == o["n_hits"], (where, n, o["n_hits"])
    assert np.array_equal(h["trait"], o["hits"]["trait"]), where
    assert np.array_equal(h["snp"], o["hits"]["snp"]), where
    rel = np.abs(h["H"] - o["hits"]["H"]) / np.maximum(np.abs(o["hits"]["H"]), 1e-300)
    assert rel.max(initial=0.0) <= H_REL, where
    assert_p(h["p"], o["hits"]["p"], where)
    return n


@pytest.fixture(scope="module")
def tiny():
    """A context whose screened-pair buffers hold 16 and 8 entries."""
    from paper_1307_3519_amd import krux
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = krux.Context(0)
    ctx.set_pair_buffer_limits(16, 8)
    yield ctx
    ctx.close()


# (K, T, M, p_missing, nan_frac): the K <= 128 kernel and the tiled kernel,
# DIAG / PLAIN / MISS3 forms, traits with NaN values as well
OVERFLOW_CASES = [(102, 70, 161, 0.05, 0.0), (48, 65, 130, 0.1, 0.02), (233, 65, 97, 0.02, 0.0),
                  (500, 40, 70, 0.01, 0.0)]


@pytest.mark.parametrize("prec", ["fp16", "int8"])
@pytest.mark.parametrize("K,T,M,pm,nan", OVERFLOW_CASES)
def test_overflow_paths_hits_and_min_p(tiny, prec, K, T, M, pm, nan):
    say("overflow hits", prec, K, T, M, pm, nan)
    x, g = _inputs(3 * K + T, T, K, M, p_missing=pm, nan_frac=nan)
    r, ts, _ = tiny.rank(_dev(x))
    p_c = 0.02
    res = tiny.test(r, ts, _dev(g), p_c=p_c, mode="hits", precision=prec, hit_capacity=1 << 15,
                    min_p=True)
    torch.cuda.synchronize()
    o = oracle.scan(x, g, p_cs=(p_c,), hits=True, min_p=True)
    # far more screened pairs than the 16 + 8 buffer entries
    assert o["n_hits"] > 24
    assert_hits(res, o, "overflow hits")
    assert_p(res["min_p"].cpu().numpy(), o["min_p"], "overflow min p")


@pytest.mark.parametrize("K,T,M,pm", [(102, 60, 120, 0.03), (233, 40, 70, 0.02)])
def test_overflow_paths_permutations(tiny, K, T, M, pm):
    say("overflow permute", K, T, M, pm)
    x, g = _inputs(5 * K + M, T, K, M, p_missing=pm)
    perms = datagen.permutations(datagen.streams(K)["perms"], 4, K)
    r, ts, _ = tiny.rank(_dev(x))
    p_cs = (0.05, 0.01, 0.001)
    gd, pd = _dev(g), _dev(perms)
    res = tiny.permute(r, ts, gd, pd, p_cs=p_cs)
    ph = tiny.permute_hits(r, ts, gd, pd, p_c=0.02, hit_capacity=1 << 14)
    torch.cuda.synchronize()
    from paper_1307_3519_amd.krux import unpack_hits
    counts = res["counts"].cpu().numpy()
    mp = res["min_p"].cpu().numpy()
    n_p, hp = unpack_hits(ph)
    tot = 0
    for i in range(perms.shape[0]):
        o = oracle.scan(x, g, p_cs=p_cs, perm=perms[i], min_p=True)
        assert np.array_equal(counts[i], o["counts"]), i
        assert_p(mp[i], o["min_p"], "overflow perm min p")
        oh = oracle.scan(x, g, p_cs=(0.02,), perm=perms[i], hits=True)
        sel = (hp["trait"] // T) == i
        assert np.array_equal(hp["trait"][sel] % T, oh["hits"]["trait"]), i
        assert np.array_equal(hp["snp"][sel], oh["hits"]["snp"]), i
        tot += oh["n_hits"]
    assert n_p == tot > 24


def test_overflow_paths_batched(tiny):
    say("overflow batched")
    M = 90
    cs = datagen.make_cohorts(M=M, Ks=(48, 102, 233), T_range=(30, 50), p_missing=0.03, seed=21)
    _check_batched(tiny, cs, M, p_c=0.02)


# ---------------------------------------------------------------- batched cohorts
@pytest.fixture(scope="module")
def kx():
    from paper_1307_3519_amd import krux
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = krux.Context(0)
    yield ctx
    ctx.close()


def _check_batched(ctx, cs, M, p_c, prec="fp16"):
    devs = []
    for c in cs:
        r, ts, _ = ctx.rank(_dev(c["expr"]))
        devs.append(dict(ranks2=r, tiesum=ts, geno=_dev(c["geno"])))
    res = ctx.test_batched(devs, M, p_c=p_c, precision=prec, hit_capacity=1 << 15, min_p=True)
    torch.cuda.synchronize()
    total = 0
    for c, rc in zip(cs, res):
        o = oracle.scan(c["expr"], c["geno"], p_cs=(p_c,), hits=True, min_p=True)
        total += assert_hits(rc, o, "cohort K=%d" % c["K"])
        assert_p(rc["min_p"].cpu().numpy(), o["min_p"], "cohort K=%d min p" % c["K"])
    assert total > 0


@pytest.mark.parametrize("prec", ["fp16", "int8"])
def test_batched_cohorts_against_oracle(kx, prec):
    # the eight sample counts of the uneven-cohort workload, 2 % missing
    # genotypes, one shared SNP panel; few traits so the oracle's per-pair
    # re-rank at K = 1000 stays within seconds
    M = 100
    say("batched cohorts", prec, M)
    cs = datagen.make_cohorts(M=M, T_range=(12, 30), p_missing=0.02, seed=17)
    assert [c["K"] for c in cs] == list(datagen.COHORT_K)
    _check_batched(kx, cs, M, p_c=0.02, prec=prec)


# ---------------------------------------------------------------- capture and growth
def test_capture_refuses_growth_and_keeps_graph_buffers():
    from paper_1307_3519_amd import krux
    say("capture growth")
    ctx = krux.Context(0)
    try:
        K, T, M, P = 102, 60, 90, 3
        x, g = _inputs(51, T, K, M)
        perms = _dev(datagen.permutations(datagen.streams(52)["perms"], P, K))
        xd, gd = _dev(x), _dev(g)
        p_cs = (0.05, 0.01)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            r, ts, _ = ctx.rank(xd)
            out = ctx.permute(r, ts, gd, perms, p_cs=p_cs)
        torch.cuda.synchronize()
        ref = out["counts"].cpu().numpy().copy(), out["min_p"].cpu().numpy().copy()
        # a call with 20x the SNPs would grow the scratch: refused under capture
        x2, g2 = _inputs(53, T, K, 20 * M)
        g2d = _dev(g2)
        graph0 = torch.cuda.CUDAGraph()
        refused = None
        with torch.cuda.graph(graph0):
            try:
                ctx.permute(r, ts, g2d, perms, p_cs=p_cs)
            except krux.KruxError as e:
                refused = str(e)
        torch.cuda.synchronize()
        assert refused is not None and "captured" in refused, refused
        del graph0
        # the same call as the eager one captures
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            ctx.permute(r, ts, gd, perms, p_cs=p_cs, out=out)
        torch.cuda.synchronize()
        # a larger eager call grows the buffers; the graph keeps its own
        big = ctx.permute(r, ts, g2d, perms, p_cs=p_cs)
        torch.cuda.synchronize()
        for i in range(P):
            o = oracle.scan(x, g2, p_cs=p_cs, perm=perms[i].cpu().numpy(), min_p=True)
            assert np.array_equal(big["counts"][i].cpu().numpy(), o["counts"]), i
        for rep in range(2):
            out["counts"].fill_(-1)
            out["min_p"].fill_(-1.0)
            graph.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out["counts"].cpu().numpy(), ref[0]), rep
            assert np.array_equal(out["min_p"].cpu().numpy(), ref[1]), rep
            ctx.permute(r, ts, g2d, perms, p_cs=p_cs)
            torch.cuda.synchronize()
    finally:
        ctx.close()
