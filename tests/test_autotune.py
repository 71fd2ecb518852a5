"""Autotuner: the chosen launch configuration is reported, persisted in the
cache file, reloaded by a fresh context, and does not change any result."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_3519_amd import datagen

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _inputs(seed, T, K, M, p_missing=0.0):
    rs = datagen.streams(seed)
    x = datagen.inject_ties(rs["ties"], datagen.to_expression(
        datagen.log_normal_z(rs["expr"], T, K)), 0.05)
    g, _ = datagen.genotypes(rs["geno"], M, K)
    g = datagen.set_missing(rs["missing"], g, p_missing)
    return x, g


@pytest.mark.parametrize("K,prec,pm", [(102, "fp16", 0.0), (77, "int8", 0.02), (233, "fp16", 0.01)])
def test_autotune_choice_persists_and_keeps_results(tmp_path, K, prec, pm):
    from paper_1307_3519_amd import krux
    print("[case] autotune", K, prec, pm, flush=True)
    T, M = 150, 700
    x, g = _inputs(50 + K, T, K, M, pm)
    cache = str(tmp_path / "tune.jsonl")
    ctx = krux.Context(0)
    try:
        r, ts, _ = ctx.rank(_dev(x))
        gd = _dev(g)
        assert ctx.tuning_of(K, prec) == dict(ring=-1, range_kb=0, grouped=-1, shape=-1)
        ms = ctx.autotune(r, ts, gd, precision=prec, cache_path=cache)
        assert ms > 0.0
        chosen = ctx.tuning_of(K, prec)
        if K <= 128:
            assert chosen["ring"] in (0, 1, 2, 3, 4) and chosen["range_kb"] in (640, 1280, 2560, 5120)
        else:
            assert chosen["grouped"] in (0, 1) and chosen["shape"] in (0, 1, 2, 3)
        res = ctx.test(r, ts, gd, p_c=0.01, precision=prec, hit_capacity=1 << 14, min_p=True)
        torch.cuda.synchronize()
        n, h = krux.unpack_hits(res)
        o = oracle.scan(x, g, p_cs=(0.01,), hits=True, min_p=True)
        assert n == o["n_hits"]
        assert np.array_equal(h["trait"], o["hits"]["trait"])
        assert np.array_equal(h["snp"], o["hits"]["snp"])
        mp = res["min_p"].cpu().numpy()
        assert np.all(np.abs(mp - o["min_p"]) <= np.maximum(1e-10 * np.abs(o["min_p"]), 1e-300))
    finally:
        ctx.close()
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"K": %d' % K in lines[0]
    ctx2 = krux.Context(0)
    try:
        ctx2.load_tuning(cache)
        assert ctx2.tuning_of(K, prec) == chosen
        assert ctx2.tuning_of(K + 1, prec) == dict(ring=-1, range_kb=0, grouped=-1, shape=-1)
    finally:
        ctx2.close()


@pytest.mark.parametrize("ring", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp16", "int8"])
@pytest.mark.parametrize("K,M", [(102, 900), (48, 1000), (17, 333)])
def test_every_pipeline_matches_oracle(tmp_path, ring, prec, K, M):
    # each SNP-stationary pipeline forced through a cache entry: register
    # double buffer, LDS ring (pipelined), LDS ring one tile at a time, two
    # per step, two SNP tiles per wave; SNP counts that leave partial blocks
    from paper_1307_3519_amd import krux
    print("[case] pipeline", ring, prec, K, M, flush=True)
    T = 300
    x, g = _inputs(70 + ring + K, T, K, M, 0.01)
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"arch": "gfx950", "K": %d, "precision": "%s", "mode": "hits", '
                     '"ring": %d, "range_kb": 640, "grouped": -1, "shape": -1, "ms": 0}\n' % (K, prec, ring))
    ctx = krux.Context(0)
    try:
        ctx.load_tuning(str(cache))
        assert ctx.tuning_of(K, prec)["ring"] == ring
        r, ts, _ = ctx.rank(_dev(x))
        res = ctx.test(r, ts, _dev(g), p_c=0.01, precision=prec, hit_capacity=1 << 14, min_p=True)
        torch.cuda.synchronize()
        n, h = krux.unpack_hits(res)
        o = oracle.scan(x, g, p_cs=(0.01,), hits=True, min_p=True)
        assert n == o["n_hits"] and n > 0
        assert np.array_equal(h["trait"], o["hits"]["trait"])
        assert np.array_equal(h["snp"], o["hits"]["snp"])
        assert np.array_equal(h["H"], o["hits"]["H"])
        mp = res["min_p"].cpu().numpy()
        assert np.all(np.abs(mp - o["min_p"]) <= np.maximum(1e-10 * np.abs(o["min_p"]), 1e-300))
    finally:
        ctx.close()


_TILE_ORACLE = {}


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", ["fp16", "int8"])
@pytest.mark.parametrize("K,T,M,pm", [(233, 300, 19000, 0.0001), (500, 520, 12000, 0.0),
                                      (150, 64, 40000, 0.001), (1000, 64, 40000, 0.00002)])
def test_every_tile_shape_matches_oracle(tmp_path, shape, prec, K, T, M, pm):
    # each tile shape of the K > 128 kernel (wide, two waves per SIMD, B side
    # from the packed codes) forced through a cache entry, with more work
    # items than resident blocks (several items per block), ragged trait
    # blocks, and a mix of complete SNP tiles and tiles with missing genotypes
    from paper_1307_3519_amd import krux
    print("[case] tile shape", shape, prec, K, T, M, pm, flush=True)
    x, g = _inputs(90 + K, T, K, M, pm)
    key = (K, T, M, pm)
    if key not in _TILE_ORACLE:
        _TILE_ORACLE[key] = oracle.scan(x, g, p_cs=(1e-3,), hits=True, min_p=True)
    o = _TILE_ORACLE[key]
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"arch": "gfx950", "K": %d, "precision": "%s", "mode": "hits", '
                     '"ring": -1, "range_kb": 0, "grouped": 1, "shape": %d, "ms": 0}\n'
                     % (K, prec, shape))
    ctx = krux.Context(0)
    try:
        ctx.load_tuning(str(cache))
        assert ctx.tuning_of(K, prec)["shape"] == shape
        r, ts, _ = ctx.rank(_dev(x))
        res = ctx.test(r, ts, _dev(g), p_c=1e-3, precision=prec, hit_capacity=1 << 16, min_p=True)
        torch.cuda.synchronize()
        n, h = krux.unpack_hits(res)
        assert n == o["n_hits"] and n > 0
        assert np.array_equal(h["trait"], o["hits"]["trait"])
        assert np.array_equal(h["snp"], o["hits"]["snp"])
        assert np.array_equal(h["H"], o["hits"]["H"])
        mp = res["min_p"].cpu().numpy()
        assert np.all(np.abs(mp - o["min_p"]) <= np.maximum(1e-10 * np.abs(o["min_p"]), 1e-300))
    finally:
        ctx.close()


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", ["fp16", "int8"])
@pytest.mark.parametrize("K,pm", [(233, 0.02), (1000, 0.02), (300, 0.0)])
def test_every_tile_shape_full_and_sums(tmp_path, shape, prec, K, pm):
    # full and sums modes run the three-column kernel over every pair
    from paper_1307_3519_amd import krux
    print("[case] tile shape full/sums", shape, prec, K, pm, flush=True)
    T, M = 70, 150
    x, g = _inputs(110 + K, T, K, M, pm)
    o = oracle.scan(x, g, full=True, sums=True)
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"arch": "gfx950", "K": %d, "precision": "%s", "mode": "hits", '
                     '"ring": -1, "range_kb": 0, "grouped": 1, "shape": %d, "ms": 0}\n'
                     % (K, prec, shape))
    ctx = krux.Context(0)
    try:
        ctx.load_tuning(str(cache))
        r, ts, _ = ctx.rank(_dev(x))
        gd = _dev(g)
        res = ctx.test(r, ts, gd, mode="sums", precision=prec)
        torch.cuda.synchronize()
        assert np.array_equal(res["sums"].cpu().numpy().astype(np.int64), o["sums"])
        res = ctx.test(r, ts, gd, mode="full", precision=prec)
        torch.cuda.synchronize()
        assert np.array_equal(res["H"].cpu().numpy(), o["H"])
    finally:
        ctx.close()
