"""HIP graph capture of the entry points that enqueue kernels only.

krux_permute (all permutations of one call), krux_test_batched (all
cohorts), krux_test in hits mode, the permuted hit lists with the FDR curve
and krux_test_noalloc enqueue only kernels on the caller's stream (no host
synchronisation, no memset: the hit sort is the library's own radix sort),
so a call can be captured once into a HIP graph and replayed as one launch.
Each replay is checked against the eager result, with unrelated eager work
of the same library between replays.
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


def _same_hits(a, b):
    from paper_1307_3519_amd.krux import unpack_hits
    na, ha = unpack_hits(a)
    nb, hb = unpack_hits(b)
    assert na == nb
    for f in ("trait", "snp", "H", "p"):
        assert np.array_equal(ha[f], hb[f]), f
    return na


def test_hits_graph_replays(kx):
    print("[case] hits graph", flush=True)
    K, T, M = 102, 400, 3000
    x, g = _inputs(61, T, K, M, 0.01)
    xd, gd = _dev(x), _dev(g)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r, ts, _ = kx.rank(xd)
        eager = kx.test(r, ts, gd, p_c=1e-3, hit_capacity=1 << 14, min_p=True)
    torch.cuda.synchronize()
    ref_mp = eager["min_p"].cpu().numpy().copy()
    out = {k: eager[k].clone() if torch.is_tensor(eager[k]) else eager[k] for k in eager}
    ref = dict(out)
    ref["n_hits_t"] = eager["n_hits_t"].clone()
    ref["hits_raw"] = eager["hits_raw"].clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rr, tt, _ = kx.rank(xd, out=(r, ts))
        kx.test(rr, tt, gd, p_c=1e-3, hit_capacity=1 << 14, min_p=True, out=out)
    torch.cuda.synchronize()
    for rep in range(3):
        out["n_hits_t"].fill_(-1)
        out["hits_raw"].fill_(0)
        out["min_p"].fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        assert _same_hits(out, ref) > 0, rep
        assert np.array_equal(out["min_p"].cpu().numpy(), ref_mp), rep
        _other_work(kx)
        torch.cuda.synchronize()


def test_fdr_curve_graph_replays(kx):
    print("[case] fdr graph", flush=True)
    K, T, M, P = 102, 200, 1500, 6
    x, g = _inputs(63, T, K, M)
    perms = _dev(datagen.permutations(datagen.streams(64)["perms"], P, K))
    xd, gd = _dev(x), _dev(g)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r, ts, _ = kx.rank(xd)
        real = kx.test(r, ts, gd, p_c=1e-3, hit_capacity=1 << 13, min_p=False)
        ph = kx.permute_hits(r, ts, gd, perms, p_c=1e-3, hit_capacity=1 << 14)
        fdr = kx.fdr_curve(real, ph, P)
    torch.cuda.synchronize()
    n_real = int(real["n_hits_t"].item())
    assert n_real > 0 and int(ph["n_hits_t"].item()) > 0
    ref = fdr[:n_real].cpu().numpy().copy()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        kx.test(r, ts, gd, p_c=1e-3, hit_capacity=1 << 13, min_p=False, out=real)
        ph2 = kx.permute_hits(r, ts, gd, perms, p_c=1e-3, hit_capacity=1 << 14)
        f2 = kx.fdr_curve(real, ph2, P)
    torch.cuda.synchronize()
    for rep in range(3):
        f2.fill_(-1.0)
        ph2["n_hits_t"].fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert _same_hits(ph2, ph) > 0, rep
        assert np.array_equal(f2[:n_real].cpu().numpy(), ref), rep
        _other_work(kx)
        torch.cuda.synchronize()


def test_noalloc_captured_on_a_fresh_context():
    # krux_test_noalloc needs no earlier eager call: its buffers are static
    from paper_1307_3519_amd import krux
    print("[case] noalloc graph", flush=True)
    ctx = krux.Context(0)
    try:
        K, T, M = 102, 500, 4000
        x, g = _inputs(9, T, K, M, 0.01)
        xd, gd = _dev(x), _dev(g)
        r, ts, _ = ctx.rank(xd)
        out = {"hits_raw": torch.empty((1 << 14) * 24, dtype=torch.uint8, device="cuda"),
               "n_hits_t": torch.zeros(1, dtype=torch.int64, device="cuda"),
               "min_p": torch.empty(T, dtype=torch.float64, device="cuda")}
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            res = ctx.test_noalloc(r, ts, gd, p_c=1e-3, hit_capacity=1 << 14, out=out)
        torch.cuda.synchronize()
        ref = ctx.test(r, ts, gd, p_c=1e-3, hit_capacity=1 << 14, min_p=True)
        torch.cuda.synchronize()
        for rep in range(3):
            out["n_hits_t"].fill_(-1)
            out["min_p"].fill_(-1.0)
            graph.replay()
            torch.cuda.synchronize()
            assert _same_hits(res, ref) > 0, rep
            assert torch.equal(res["min_p"], ref["min_p"]), rep
            # other work on the static array between replays
            ctx.test_noalloc(r, ts, gd[:500], p_c=1e-2, hit_capacity=1 << 10)
            torch.cuda.synchronize()
    finally:
        ctx.close()
