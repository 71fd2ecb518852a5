"""HIP graph capture of the batched entry points.

krux_permute (all permutations of one call) and krux_test_batched (all
cohorts) enqueue only kernels on the caller's stream, with no host
synchronisation, so a call can be captured once into a HIP graph and the
graph replayed as one launch.  Each replay is checked against the eager
result, with unrelated eager work of the same library between replays.
"""
import numpy as np
import pytest
import torch

from paper_1307_3519_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kx():
    from paper_1307_3519_amd import krux
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = krux.Context(0)
    yield ctx
    ctx.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _inputs(seed, T, K, M, p_missing=0.0):
    rs = datagen.streams(seed)
    x = datagen.inject_ties(rs["ties"], datagen.to_expression(
        datagen.log_normal_z(rs["expr"], T, K)), 0.05)
    g, _ = datagen.genotypes(rs["geno"], M, K)
    g = datagen.set_missing(rs["missing"], g, p_missing)
    return x, g


def _other_work(kx):
    x, g = _inputs(77, 50, 60, 70, 0.05)
    r, ts, _ = kx.rank(_dev(x))
    kx.test(r, ts, _dev(g), p_c=0.01, hit_capacity=1024)


def test_permute_graph_replays(kx):
    print("[case] permute graph", flush=True)
    K, T, M, P = 102, 300, 250, 12
    x, g = _inputs(41, T, K, M)
    perms = datagen.permutations(datagen.streams(43)["perms"], P, K)
    xd, gd, pd = _dev(x), _dev(g), _dev(perms)
    r, ts, _ = kx.rank(xd)
    p_cs = (0.05, 0.01, 0.001)
    out = {"counts": torch.empty((P, 3), dtype=torch.int64, device="cuda"),
           "min_p": torch.empty((P, T), dtype=torch.float64, device="cuda")}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):            # eager call: grows the context's buffers
        kx.permute(r, ts, gd, pd, p_cs=p_cs, out=out)
    torch.cuda.synchronize()
    ref_counts = out["counts"].cpu().numpy().copy()
    ref_minp = out["min_p"].cpu().numpy().copy()
    assert ref_counts[:, 0].sum() > 0
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        kx.permute(r, ts, gd, pd, p_cs=p_cs, out=out)
    torch.cuda.synchronize()
    for rep in range(3):
        out["counts"].fill_(-1)
        out["min_p"].fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out["counts"].cpu().numpy(), ref_counts), rep
        assert np.array_equal(out["min_p"].cpu().numpy(), ref_minp), rep
        _other_work(kx)
        torch.cuda.synchronize()


def test_batched_cohorts_graph_replays(kx):
    print("[case] batched cohorts graph", flush=True)
    from paper_1307_3519_amd.krux import unpack_hits
    M = 300
    cs = datagen.make_cohorts(M=M, Ks=(48, 102, 233), T_range=(40, 90), p_missing=0.02, seed=9)
    devs = []
    for c in cs:
        r, ts, _ = kx.rank(_dev(c["expr"]))
        devs.append(dict(ranks2=r, tiesum=ts, geno=_dev(c["geno"])))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        eager = kx.test_batched(devs, M, p_c=0.01, hit_capacity=4096, min_p=True)
    torch.cuda.synchronize()
    ref = [(unpack_hits(e), e["min_p"].cpu().numpy().copy()) for e in eager]
    assert sum(h[0][0] for h in ref) > 0
    bufs = kx.test_batched_buffers(devs, hit_capacity=4096, min_p=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        kx.test_batched(devs, M, p_c=0.01, hit_capacity=4096, min_p=True, out=bufs)
    torch.cuda.synchronize()
    for rep in range(3):
        for b in bufs:
            b["n_hits_t"].fill_(-1)
            b["min_p"].fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        for b, ((n, h), mp) in zip(bufs, ref):
            n2, h2 = unpack_hits(b)
            assert n2 == n, rep
            assert np.array_equal(h2["trait"], h["trait"]) and np.array_equal(h2["snp"], h["snp"])
            assert np.array_equal(h2["H"], h["H"])
            assert np.array_equal(b["min_p"].cpu().numpy(), mp)
        _other_work(kx)
        torch.cuda.synchronize()
