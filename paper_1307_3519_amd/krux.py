"""Thin ctypes binding of libkrux.so (C ABI in include/krux.h).

Only argument marshalling happens here: torch tensors provide device memory
and the current HIP stream; every step of the computation runs in the
library's gfx950 kernels.  There is no CPU fallback: if the library is
missing or no gfx950 GPU is present the calls raise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# KRUX_LIBRARY may name another build of the same library (e.g. a tuning build)
LIB_PATH = os.environ.get("KRUX_LIBRARY") or os.path.join(_HERE, "libkrux.so")

KRUX_OK = 0
MODE_HITS, MODE_FULL, MODE_SUMS = 0, 1, 2
PREC_FP16, PREC_INT8, PREC_FP64 = 0, 1, 2
_PREC = {"fp16": PREC_FP16, "int8": PREC_INT8, "fp64": PREC_FP64}
_MODE = {"hits": MODE_HITS, "full": MODE_FULL, "sums": MODE_SUMS}

EXPORTS = ("krux_create", "krux_destroy", "krux_last_error", "krux_threshold",
           "krux_rank", "krux_test", "krux_permute", "krux_permute_hits", "krux_fdr_curve",
           "krux_test_grouped", "krux_test_multi",
           "krux_test_batched",
           "krux_timer_start", "krux_timer_read", "krux_autotune", "krux_load_tuning",
           "krux_tuning_of", "krux_set_pair_buffer_limits", "krux_test_noalloc")


class KruxError(RuntimeError):
    pass


class Hit(ctypes.Structure):
    _fields_ = [("trait", ctypes.c_int32), ("snp", ctypes.c_int32),
                ("H", ctypes.c_double), ("p", ctypes.c_double)]


class Cohort(ctypes.Structure):
    _fields_ = [("ranks2", ctypes.c_void_p), ("tiesum", ctypes.c_void_p),
                ("T", ctypes.c_int64), ("K", ctypes.c_int32),
                ("geno", ctypes.c_void_p), ("ld_geno", ctypes.c_int64),
                ("hits", ctypes.c_void_p), ("hit_capacity", ctypes.c_int64),
                ("n_hits", ctypes.c_void_p), ("min_p", ctypes.c_void_p)]


_lib = None


def library():
    """Load libkrux.so from the package directory (build it first with
    ``python -m paper_1307_3519_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise KruxError("libkrux.so is not built (python -m paper_1307_3519_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.krux_create.restype = ctypes.c_int
    lib.krux_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    lib.krux_destroy.restype = None
    lib.krux_destroy.argtypes = [P]
    lib.krux_last_error.restype = ctypes.c_char_p
    lib.krux_last_error.argtypes = [P]
    lib.krux_threshold.restype = ctypes.c_int
    lib.krux_threshold.argtypes = [dbl, i32, ctypes.POINTER(ctypes.c_double)]
    lib.krux_rank.restype = ctypes.c_int
    lib.krux_rank.argtypes = [P, P, i64, i32, i64, P, P, P, P]
    lib.krux_test.restype = ctypes.c_int
    lib.krux_test.argtypes = [P, P, P, i64, i32, P, i64, i64, i64, dbl, i32, i32,
                              P, i64, P, P, P, P, P, P]
    lib.krux_test_noalloc.restype = ctypes.c_int
    lib.krux_test_noalloc.argtypes = lib.krux_test.argtypes
    lib.krux_permute.restype = ctypes.c_int
    lib.krux_permute.argtypes = [P, P, P, i64, i32, P, i64, i64, P, i32, P, i32, P, P, P]
    lib.krux_test_batched.restype = ctypes.c_int
    lib.krux_test_multi.restype = ctypes.c_int
    lib.krux_test_multi.argtypes = [P, P, P, i64, i32, P, i64, i64, i32, i64, dbl, i32, P, i64,
                                    P, P, P, P, P]
    lib.krux_test_grouped.restype = ctypes.c_int
    lib.krux_test_grouped.argtypes = [P, P, P, i64, i32, P, i64, i64, i64, dbl, i32, i64, P, i64,
                                      P, P, P]
    lib.krux_permute_hits.restype = ctypes.c_int
    lib.krux_permute_hits.argtypes = [P, P, P, i64, i32, P, i64, i64, P, i32, dbl, P, i64, P, P]
    lib.krux_fdr_curve.restype = ctypes.c_int
    lib.krux_fdr_curve.argtypes = [P, P, P, i64, P, P, i64, i32, P, P]
    lib.krux_test_batched.argtypes = [P, P, i32, i64, dbl, i32, P]
    lib.krux_timer_start.restype = ctypes.c_int
    lib.krux_timer_start.argtypes = [P]
    lib.krux_timer_read.restype = ctypes.c_int
    lib.krux_timer_read.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
    lib.krux_autotune.restype = ctypes.c_int
    lib.krux_autotune.argtypes = [P, P, P, i64, i32, P, i64, i64, i32, ctypes.c_char_p,
                                  ctypes.POINTER(ctypes.c_double), P]
    lib.krux_load_tuning.restype = ctypes.c_int
    lib.krux_load_tuning.argtypes = [P, ctypes.c_char_p]
    lib.krux_set_pair_buffer_limits.restype = ctypes.c_int
    lib.krux_set_pair_buffer_limits.argtypes = [P, i64, i64]
    lib.krux_tuning_of.restype = ctypes.c_int
    lib.krux_tuning_of.argtypes = [P, i32, i32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def threshold(p_c, df):
    h = ctypes.c_double()
    lib = library()
    st = lib.krux_threshold(float(p_c), int(df), ctypes.byref(h))
    if st != KRUX_OK:
        raise KruxError(lib.krux_last_error(None).decode())
    return h.value


class Context:
    """A library context on one device (owns the scratch memory)."""

    def __init__(self, device=0):
        self.lib = library()
        h = ctypes.c_void_p()
        st = self.lib.krux_create(ctypes.byref(h), int(device))
        if st != KRUX_OK:
            raise KruxError(self.lib.krux_last_error(None).decode())
        self.h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if self.h:
            self.lib.krux_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != KRUX_OK:
            raise KruxError("status %d: %s" % (st, self.lib.krux_last_error(self.h).decode()))

    # ------------------------------------------------------------------ timer
    def timer_start(self):
        """Bracket every fused scan kernel launch of the main pass with events."""
        self._check(self.lib.krux_timer_start(self.h))

    def timer_read(self):
        """-> (summed kernel milliseconds, number of launches); stops the timer."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.krux_timer_read(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def set_pair_buffer_limits(self, candidates=0, missing_pairs=0):
        """Caps (entries, 0 = built in) on the screened-pair buffers; pairs
        beyond them are evaluated inside the scan kernels."""
        self._check(self.lib.krux_set_pair_buffer_limits(self.h, int(candidates),
                                                         int(missing_pairs)))

    # ------------------------------------------------------------------ tuning
    def autotune(self, ranks2, tiesum, geno, precision="fp16", cache_path=None):
        """Times every launch configuration for (K, precision) on these inputs
        and keeps the fastest in the context; -> best milliseconds per call."""
        T, K = ranks2.shape
        M = geno.shape[0]
        ms = ctypes.c_double()
        self._check(self.lib.krux_autotune(
            self.h, _ptr(ranks2), _ptr(tiesum), T, K, _ptr(geno), M,
            geno.stride(0) if M else K, _PREC[precision],
            cache_path.encode() if cache_path else None, ctypes.byref(ms), _stream()))
        return ms.value

    def load_tuning(self, cache_path):
        self._check(self.lib.krux_load_tuning(self.h, cache_path.encode()))

    def tuning_of(self, K, precision="fp16"):
        """-> dict(ring, range_kb, grouped, shape) in use for (K, precision)."""
        r, kb, g, sh = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.krux_tuning_of(self.h, K, _PREC[precision], ctypes.byref(r),
                                            ctypes.byref(kb), ctypes.byref(g), ctypes.byref(sh)))
        return dict(ring=r.value, range_kb=kb.value, grouped=g.value, shape=sh.value)

    # ------------------------------------------------------------------ rank
    def rank(self, expr, out=None):
        """expr: (T, K) float32 cuda tensor (row-contiguous, any row stride)
        -> ranks2 (T, K) int16, tiesum (T,) int64, nvalid (T,) int32.
        `out` may pass (ranks2, tiesum[, nvalid]) buffers."""
        assert expr.is_cuda and expr.dtype == torch.float32 and expr.dim() == 2
        assert expr.stride(1) == 1
        T, K = expr.shape
        if out is not None:
            r, ts = out[0], out[1]
            nv = out[2] if len(out) > 2 else None
            assert r.shape == (T, K) and r.dtype == torch.int16 and r.is_contiguous()
            assert ts.shape == (T,) and ts.dtype == torch.int64
        else:
            r = torch.empty((T, K), dtype=torch.int16, device=expr.device)
            ts = torch.empty(T, dtype=torch.int64, device=expr.device)
            nv = torch.empty(T, dtype=torch.int32, device=expr.device)
        self._check(self.lib.krux_rank(self.h, _ptr(expr), T, K, expr.stride(0) if T else K,
                                       _ptr(r), _ptr(ts), _ptr(nv), _stream()))
        return r, ts, nv

    # ------------------------------------------------------------------ test
    def test(self, ranks2, tiesum, geno, p_c=1e-5, mode="hits", precision="fp16",
             hit_capacity=1 << 16, min_p=True, snp_base=0, out=None):
        """One scan of every trait against every SNP of geno (M, K) int8.

        hits mode -> dict(n_hits, hits (structured tensor view), min_p)
        full mode -> dict(H, p) (T, M) float64
        sums mode -> dict(sums) (3, T, M) int32
        `out` may pass preallocated buffers (same keys) to avoid allocation.
        """
        return self._test(self.lib.krux_test, ranks2, tiesum, geno, p_c, mode, precision,
                          hit_capacity, min_p, snp_base, out)

    def test_noalloc(self, ranks2, tiesum, geno, p_c=1e-5, mode="hits", precision="fp16",
                     hit_capacity=1 << 16, min_p=True, snp_base=0, out=None):
        """As test(), through krux_test_noalloc: the library allocates no
        device memory (its working buffers come from a static array)."""
        return self._test(self.lib.krux_test_noalloc, ranks2, tiesum, geno, p_c, mode,
                          precision, hit_capacity, min_p, snp_base, out)

    def _test(self, fn, ranks2, tiesum, geno, p_c, mode, precision, hit_capacity, min_p,
              snp_base, out):
        T, K = ranks2.shape
        M = geno.shape[0]
        assert geno.dtype == torch.int8 and geno.dim() == 2 and geno.shape[1] == K
        assert M == 0 or geno.stride(1) == 1
        dev = ranks2.device
        out = dict(out or {})
        m = _MODE[mode]
        pr = _PREC[precision]
        hits = nh = mp = H = p = sums = None
        if m == MODE_HITS:
            hits = out.get("hits_raw")
            if hits is None or hits.numel() < hit_capacity * 24:
                hits = torch.empty(max(hit_capacity, 1) * 24, dtype=torch.uint8, device=dev)
            nh = out.get("n_hits_t")
            if nh is None:
                nh = torch.zeros(1, dtype=torch.int64, device=dev)
            if min_p:
                mp = out.get("min_p")
                if mp is None:
                    mp = torch.empty(T, dtype=torch.float64, device=dev)
        elif m == MODE_FULL:
            H = out.get("H")
            p = out.get("p")
            if H is None:
                H = torch.empty((T, M), dtype=torch.float64, device=dev)
            if p is None:
                p = torch.empty((T, M), dtype=torch.float64, device=dev)
        else:
            sums = out.get("sums")
            if sums is None:
                sums = torch.empty((3, T, M), dtype=torch.int32, device=dev)
        self._check(fn(
            self.h, _ptr(ranks2), _ptr(tiesum), T, K, _ptr(geno), M,
            geno.stride(0) if M else K, int(snp_base), float(p_c), m, pr,
            _ptr(hits), int(hit_capacity) if m == MODE_HITS else 0, _ptr(nh), _ptr(mp),
            _ptr(H), _ptr(p), _ptr(sums), _stream()))
        if m == MODE_HITS:
            return dict(hits_raw=hits, n_hits_t=nh, min_p=mp, hit_capacity=hit_capacity)
        if m == MODE_FULL:
            return dict(H=H, p=p)
        return dict(sums=sums)

    def test_grouped(self, ranks2, tiesum, geno, p_c=1e-5, precision="fp16", min_group=256,
                     hit_capacity=1 << 16, min_p=True, snp_base=0):
        """As test() in hits mode, with SNPs grouped by missing-genotype pattern."""
        T, K = ranks2.shape
        M = geno.shape[0]
        assert geno.dtype == torch.int8 and geno.dim() == 2 and geno.shape[1] == K
        assert M == 0 or geno.stride(1) == 1
        dev = ranks2.device
        hits = torch.empty(max(hit_capacity, 1) * 24, dtype=torch.uint8, device=dev)
        nh = torch.zeros(1, dtype=torch.int64, device=dev)
        mp = torch.empty(T, dtype=torch.float64, device=dev) if min_p else None
        self._check(self.lib.krux_test_grouped(
            self.h, _ptr(ranks2), _ptr(tiesum), T, K, _ptr(geno), M,
            geno.stride(0) if M else K, int(snp_base), float(p_c), _PREC[precision],
            int(min_group), _ptr(hits), int(hit_capacity), _ptr(nh), _ptr(mp), _stream()))
        return dict(hits_raw=hits, n_hits_t=nh, min_p=mp, hit_capacity=hit_capacity)

    def test_multi(self, ranks2, tiesum, geno, n_classes, p_c=1e-5, mode="hits",
                   hit_capacity=1 << 16, snp_base=0, min_p=True):
        """Multi-allelic markers (codes 0..n_classes-1): hits mode -> dict as
        test(); full mode -> dict(H, p) (T, M) float64."""
        T, K = ranks2.shape
        M = geno.shape[0]
        assert geno.dtype == torch.int8 and geno.dim() == 2 and geno.shape[1] == K
        assert M == 0 or geno.stride(1) == 1
        dev = ranks2.device
        m = _MODE[mode]
        hits = nh = H = p = mp = None
        if m == MODE_HITS:
            hits = torch.empty(max(hit_capacity, 1) * 24, dtype=torch.uint8, device=dev)
            nh = torch.zeros(1, dtype=torch.int64, device=dev)
            if min_p:
                mp = torch.empty(T, dtype=torch.float64, device=dev)
        else:
            H = torch.empty((T, M), dtype=torch.float64, device=dev)
            p = torch.empty((T, M), dtype=torch.float64, device=dev)
        self._check(self.lib.krux_test_multi(
            self.h, _ptr(ranks2), _ptr(tiesum), T, K, _ptr(geno), M,
            geno.stride(0) if M else K, int(n_classes), int(snp_base), float(p_c), m,
            _ptr(hits), int(hit_capacity) if m == MODE_HITS else 0, _ptr(nh), _ptr(mp), _ptr(H),
            _ptr(p), _stream()))
        if m == MODE_HITS:
            return dict(hits_raw=hits, n_hits_t=nh, min_p=mp, hit_capacity=hit_capacity)
        return dict(H=H, p=p)

    # ------------------------------------------------------------------ permute
    def permute(self, ranks2, tiesum, geno, perms, p_cs=(1e-4, 1e-5, 1e-6), min_p=True,
                out=None):
        """perms (P, K) int32 cuda -> dict(counts (P, n_thr) int64, min_p (P, T))."""
        T, K = ranks2.shape
        M = geno.shape[0]
        P = perms.shape[0]
        dev = ranks2.device
        out = dict(out or {})
        counts = out.get("counts")
        if counts is None:
            counts = torch.empty((P, len(p_cs)), dtype=torch.int64, device=dev)
        mp = None
        if min_p:
            mp = out.get("min_p")
            if mp is None:
                mp = torch.empty((P, T), dtype=torch.float64, device=dev)
        pcs = (ctypes.c_double * len(p_cs))(*[float(x) for x in p_cs])
        self._check(self.lib.krux_permute(
            self.h, _ptr(ranks2), _ptr(tiesum), T, K, _ptr(geno), M,
            geno.stride(0) if M else K, _ptr(perms), P, pcs, len(p_cs), _ptr(counts), _ptr(mp),
            _stream()))
        return dict(counts=counts, min_p=mp)

    def permute_hits(self, ranks2, tiesum, geno, perms, p_c=1e-5, hit_capacity=1 << 20):
        """Hit list of the permuted data, rows perm * T + trait in the trait
        field -> dict as test() in hits mode."""
        T, K = ranks2.shape
        M = geno.shape[0]
        P = perms.shape[0]
        dev = ranks2.device
        hits = torch.empty(max(hit_capacity, 1) * 24, dtype=torch.uint8, device=dev)
        nh = torch.zeros(1, dtype=torch.int64, device=dev)
        self._check(self.lib.krux_permute_hits(
            self.h, _ptr(ranks2), _ptr(tiesum), T, K, _ptr(geno), M,
            geno.stride(0) if M else K, _ptr(perms), P, float(p_c), _ptr(hits),
            int(hit_capacity), _ptr(nh), _stream()))
        return dict(hits_raw=hits, n_hits_t=nh, min_p=None, hit_capacity=hit_capacity)

    def fdr_curve(self, real, perm, P):
        """Empirical FDR at the p of every real hit: real from test() (hits
        mode), perm from permute_hits() over P permutations -> (real_cap,)
        float64 tensor, valid up to the real hit count."""
        dev = real["hits_raw"].device
        fdr = torch.full((max(real["hit_capacity"], 1),), float("nan"), dtype=torch.float64,
                         device=dev)
        self._check(self.lib.krux_fdr_curve(
            self.h, _ptr(real["hits_raw"]), _ptr(real["n_hits_t"]), int(real["hit_capacity"]),
            _ptr(perm["hits_raw"]), _ptr(perm["n_hits_t"]), int(perm["hit_capacity"]), int(P),
            _ptr(fdr), _stream()))
        return fdr

    # ------------------------------------------------------------------ cohorts
    def test_batched_buffers(self, cohorts, hit_capacity=1 << 16, min_p=False):
        """Output buffers of test_batched (one dict per cohort), for `out`."""
        res = []
        for c in cohorts:
            T = c["ranks2"].shape[0]
            dev = c["ranks2"].device
            res.append(dict(
                hits_raw=torch.empty(max(hit_capacity, 1) * 24, dtype=torch.uint8, device=dev),
                n_hits_t=torch.zeros(1, dtype=torch.int64, device=dev),
                min_p=torch.empty(T, dtype=torch.float64, device=dev) if min_p else None,
                hit_capacity=hit_capacity))
        return res

    def test_batched(self, cohorts, M, p_c=1e-5, precision="fp16", hit_capacity=1 << 16,
                     min_p=False, out=None):
        """cohorts: list of dicts with ranks2, tiesum, geno (device tensors).
        Returns a list of result dicts (hits_raw, n_hits_t, min_p); `out` may
        pass the buffers of test_batched_buffers."""
        res = out if out is not None else self.test_batched_buffers(cohorts, hit_capacity, min_p)
        arr = (Cohort * len(cohorts))()
        for i, (c, b) in enumerate(zip(cohorts, res)):
            T, K = c["ranks2"].shape
            mp = b["min_p"]
            arr[i] = Cohort(c["ranks2"].data_ptr(), c["tiesum"].data_ptr(), T, K,
                            c["geno"].data_ptr(), c["geno"].stride(0), b["hits_raw"].data_ptr(),
                            b["hit_capacity"], b["n_hits_t"].data_ptr(),
                            mp.data_ptr() if mp is not None else None)
        self._check(self.lib.krux_test_batched(self.h, ctypes.cast(arr, ctypes.c_void_p),
                                               len(cohorts), int(M), float(p_c),
                                               _PREC[precision], _stream()))
        return res


def unpack_hits(res):
    """Host copy of a hits-mode result: (n_hits, dict of numpy arrays)."""
    import numpy as np
    n = int(res["n_hits_t"].item())
    k = min(n, res["hit_capacity"])
    raw = res["hits_raw"][: k * 24].cpu().numpy()
    dt = np.dtype([("trait", "<i4"), ("snp", "<i4"), ("H", "<f8"), ("p", "<f8")])
    rec = raw.view(dt) if k else np.zeros(0, dt)
    return n, dict(trait=rec["trait"].copy(), snp=rec["snp"].copy(), H=rec["H"].copy(),
                   p=rec["p"].copy())
