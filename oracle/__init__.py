"""CPU oracle for the Kruskal-Wallis SNP x trait scan (kruX, arXiv:1307.3519).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It is a plain,
slow, obviously-correct reference (C with OpenMP, fp64, exact integer rank
sums, exact rational H) and shares no code with the GPU library.

Functions follow the paper's sections:
  rank()       -- ranks per trait and the tie term (Implementation: input
                  data; handling tied data)
  one_pair()   -- eq. (2) divided by the tie factor, empty groups dropped
  threshold()  -- statistic threshold for a p-value threshold (P-value
                  calculation)
  pvalue()     -- chi-square tail for df = 1, 2
  scan()       -- every pair: full H/p matrices, group sums, hit lists,
                  per-threshold counts, per-trait minimum p, optional column
                  permutation of the rank matrix (empirical FDR)
  fdr_curve()  -- empirical FDR at given p-values from real and permuted
                  p-values (P-value calculation and empirical FDR correction)
Missing genotypes (code -1) remove the sample from that pair and the ranks
are recomputed over the remaining samples (handling missing values).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "krux_oracle.c")
_LIB = os.path.join(_HERE, "libkrux_oracle.so")
_lib = None


def build(force=False):
    """Compile the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def use_library(path=None):
    """Load the oracle from `path` (a variant built by the tests, e.g. with a
    planted mistake) or, with None, from the default build."""
    global _lib
    _lib = None
    _load(path)


def _load(path=None):
    global _lib
    if _lib is None:
        if path is None:
            build()
        lib = ctypes.CDLL(path or _LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.restype = None
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_rational_to_double_parts.restype = dbl
        lib.oracle_rational_to_double_parts.argtypes = [ctypes.c_uint64] * 4
        lib.oracle_pvalue.restype = dbl
        lib.oracle_pvalue.argtypes = [dbl, ctypes.c_int]
        lib.oracle_threshold.restype = dbl
        lib.oracle_threshold.argtypes = [dbl, ctypes.c_int]
        lib.oracle_rank.restype = None
        lib.oracle_rank.argtypes = [P, i64, i32, i64, P, P, P]
        lib.oracle_one_pair.restype = None
        lib.oracle_one_pair.argtypes = [P, P, i32, P, P, P, P, P, P, P]
        lib.oracle_scan.restype = ctypes.c_int
        lib.oracle_scan.argtypes = [P, i64, i32, i64, P, i64, i64, P, P, i32,
                                    P, P, P, P, P, P, P, P, P, i64, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads():
    return _load().oracle_num_threads()


def set_num_threads(n):
    """Threads of later scans (OpenMP)."""
    _load().oracle_set_num_threads(int(n))


def rational_to_double(num, den):
    """Nearest double to the rational num/den (non-negative ints < 2**128)."""
    m = (1 << 64) - 1
    return _load().oracle_rational_to_double_parts(num >> 64, num & m, den >> 64, den & m)


def pvalue(H, df):
    return _load().oracle_pvalue(float(H), int(df))


def threshold(p_c, df):
    """Largest double h >= 0 with pvalue(h, df) >= p_c."""
    return _load().oracle_threshold(float(p_c), int(df))


def rank(expr):
    """expr: (T, K) float32 -> (ranks2 int32 (T, K), tiesum int64 (T,), nvalid int32 (T,))."""
    expr = np.ascontiguousarray(expr, dtype=np.float32)
    T, K = expr.shape
    r = np.empty((T, K), np.int32)
    ts = np.empty(T, np.int64)
    nv = np.empty(T, np.int32)
    _load().oracle_rank(_ptr(expr), T, K, K, _ptr(r), _ptr(ts), _ptr(nv))
    return r, ts, nv


def one_pair(x, g):
    """One trait row x (K,) and genotype row g (K,) -> dict."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    g = np.ascontiguousarray(g, dtype=np.int8)
    K = x.shape[0]
    H = np.zeros(1); p = np.zeros(1)
    df = np.zeros(1, np.int32); n = np.zeros(3, np.int32)
    s2 = np.zeros(3, np.int64); ts = np.zeros(1, np.int64); ko = np.zeros(1, np.int32)
    _load().oracle_one_pair(_ptr(x), _ptr(g), K, _ptr(H), _ptr(p), _ptr(df),
                            _ptr(n), _ptr(s2), _ptr(ts), _ptr(ko))
    return dict(H=float(H[0]), p=float(p[0]), df=int(df[0]), n=n.copy(),
                s2=s2.copy(), tiesum=int(ts[0]), kobs=int(ko[0]))


def scan(expr, geno, p_cs=(), perm=None, full=False, sums=False,
         min_p=False, hits=False, hit_cap=None):
    """Every SNP x trait pair.

    expr (T, K) float32; geno (M, K) int8 codes {0,1,2,-1}; p_cs: p-value
    thresholds (hits are taken at p_cs[0]); perm: optional (K,) int column
    permutation of the rank matrix.  Returns a dict with the requested parts:
    H, p (T, M) float64; sums (3, T, M) int64 doubled group rank sums;
    counts (len(p_cs),) int64; min_p (T,); hits: structured arrays
    trait, snp, H, p in (trait, snp) order; n_hits.
    """
    lib = _load()
    expr = np.ascontiguousarray(expr, dtype=np.float32)
    geno = np.ascontiguousarray(geno, dtype=np.int8)
    T, K = expr.shape
    M = geno.shape[0]
    assert geno.shape[1] == K
    n_thr = len(p_cs)
    Hc = np.array([[threshold(pc, 1), threshold(pc, 2)] for pc in p_cs],
                  dtype=np.float64).reshape(-1)
    out = {}
    H = np.empty((T, M)) if full else None
    p = np.empty((T, M)) if full else None
    S = np.empty((3, T, M), np.int64) if sums else None
    counts = np.zeros(max(n_thr, 1), np.int64)
    mp = np.empty(T) if min_p else None
    if perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        assert perm.shape == (K,) and np.array_equal(np.sort(perm), np.arange(K))
    nh = np.zeros(1, np.int64)
    if hits:
        if hit_cap is None:
            # first call counts, second call fills
            lib.oracle_scan(_ptr(expr), T, K, K, _ptr(geno), M, K, _ptr(perm),
                            _ptr(Hc), n_thr, None, None, None, None, None,
                            None, None, None, None, 0, _ptr(nh))
            hit_cap = int(nh[0])
        ht = np.empty(hit_cap, np.int32); hs = np.empty(hit_cap, np.int32)
        hH = np.empty(hit_cap); hp = np.empty(hit_cap)
    else:
        ht = hs = hH = hp = None
        hit_cap = 0
    lib.oracle_scan(_ptr(expr), T, K, K, _ptr(geno), M, K, _ptr(perm),
                    _ptr(Hc), n_thr, _ptr(H), _ptr(p), _ptr(S),
                    _ptr(counts) if n_thr else None, _ptr(mp),
                    _ptr(ht), _ptr(hs), _ptr(hH), _ptr(hp), hit_cap,
                    _ptr(nh) if hits else None)
    if full:
        out["H"], out["p"] = H, p
    if sums:
        out["sums"] = S
    if n_thr:
        out["counts"] = counts[:n_thr]
        out["Hc"] = Hc.reshape(n_thr, 2)
    if min_p:
        out["min_p"] = mp
    if hits:
        n = int(nh[0])
        k = min(n, hit_cap)
        out["n_hits"] = n
        out["hits"] = dict(trait=ht[:k], snp=hs[:k], H=hH[:k], p=hp[:k])
    return out


def fdr_curve(real_p, perm_p, P, at=None):
    """Empirical FDR (P-value calculation and empirical FDR correction): for a
    value q, the number of permuted associations with p <= q averaged over
    the P permutations, divided by the number of real associations with
    p <= q.  Evaluated at each q of `at` (default: the real p-values), by
    plain counting; the ratio is formed as count / (P * count) in double."""
    real_p = np.asarray(real_p, np.float64)
    perm_p = np.asarray(perm_p, np.float64)
    at = real_p if at is None else np.asarray(at, np.float64)
    out = np.empty(len(at))
    for i, q in enumerate(at):
        n_perm = int(np.count_nonzero(perm_p <= q))
        n_real = int(np.count_nonzero(real_p <= q))
        out[i] = n_perm / (float(P) * float(n_real)) if n_real else float("nan")
    return out
