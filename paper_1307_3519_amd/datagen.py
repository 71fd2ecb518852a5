"""Seeded synthetic inputs shaped like the paper's human eQTL workload.

This module only draws random inputs; it holds none of the test's
arithmetic, and both the GPU path and the CPU oracle are fed from it.

The paper's data (102 whole-blood samples, ~20k expression traits, ~530k SNPs
with MAF > 5%, no missing values, in Hardy-Weinberg equilibrium; Results,
"Validation data") is not available, so these generators stand in for it:

  expression  z ~ N(0, 1), value = float32(exp(z)) (log-normal(0, 1)); then
              round(tie_frac * K) distinct positions per row are overwritten
              with the value of a uniformly chosen other (non-target)
              position of the same row, which forces ties;
  genotypes   per SNP a minor-allele frequency q ~ U[0.05, 0.5] and codes
              G ~ Binomial(2, q) (Hardy-Weinberg), int8 in {0, 1, 2};
  planted     distinct traits each paired with one SNP whose three genotype
              classes all have >= 2 samples; a shift delta ~ U[0.5, 2.0] SD
              is added to z (before exp and before the ties) under an
              additive (delta*g), dominant (delta*[g>=1]) or single-group
              outlier (delta*[g == smallest class]) model;
  missing     each genotype independently set to -1 with probability p;
  permutations  rows of independent uniform permutations of range(K).

Every stream comes from numpy's PCG64 seeded by SeedSequence(seed).spawn(),
one child per purpose, so each part is reproducible on its own.
"""
import numpy as np

_STREAMS = ("expr", "ties", "geno", "plant", "perms", "missing", "cohort", "nan")


def streams(seed):
    kids = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    return {name: np.random.Generator(np.random.PCG64(s)) for name, s in zip(_STREAMS, kids)}


def log_normal_z(rng, T, K):
    return rng.standard_normal((T, K))


def to_expression(z):
    return np.exp(z).astype(np.float32)


def inject_ties(rng, x, tie_frac=0.05):
    """Overwrite round(tie_frac*K) distinct positions of every row with the
    value of a uniformly chosen non-target position of the same row."""
    T, K = x.shape
    n_t = int(round(tie_frac * K))
    if n_t == 0 or K < 2:
        return x
    n_t = min(n_t, K - 1)
    keys = rng.random((T, K))
    order = np.argsort(keys, axis=1)
    targets = order[:, :n_t]
    others = order[:, n_t:]
    pick = rng.integers(0, K - n_t, size=(T, n_t))
    src = np.take_along_axis(others, pick, axis=1)
    rows = np.arange(T)[:, None]
    x[rows, targets] = x[rows, src]
    return x


def genotypes(rng, M, K, maf_lo=0.05, maf_hi=0.5, q=None):
    if q is None:
        q = rng.uniform(maf_lo, maf_hi, size=M)
    g = rng.binomial(2, q[:, None], size=(M, K)).astype(np.int8)
    return g, q


def set_missing(rng, g, p_missing):
    if p_missing <= 0:
        return g
    mask = rng.random(g.shape) < p_missing
    g = g.copy()
    g[mask] = -1
    return g


def set_missing_samples(rng, g, sample_sets, fracs):
    """Sample-structured missing genotypes (a failed sample): for each set of
    samples and its fraction, each SNP, with that probability, has every
    sample of the set missing (-1).  Later sets overwrite earlier ones."""
    g = g.copy()
    for samples, frac in zip(sample_sets, fracs):
        rows = rng.random(g.shape[0]) < frac
        g[np.ix_(rows, np.asarray(samples, dtype=np.int64))] = -1
    return g


def set_nan_expression(rng, x, trait_frac, max_per_trait):
    """Missing expression values: each trait, with probability trait_frac,
    gets between 1 and max_per_trait NaN entries at distinct samples."""
    T, K = x.shape
    x = x.copy()
    rows = np.flatnonzero(rng.random(T) < trait_frac)
    for t in rows:
        n = int(rng.integers(1, max_per_trait + 1))
        x[t, rng.choice(K, size=min(n, K), replace=False)] = np.nan
    return x


def plant(rng, z, g, n_pairs, min_class=2):
    """Add genotype-dependent shifts to n_pairs distinct traits of z (in place).
    Returns an int64 array (n_pairs, 3): trait, snp, model (0 additive,
    1 dominant, 2 single-group outlier)."""
    T = z.shape[0]
    M = g.shape[0]
    n_pairs = min(n_pairs, T)
    traits = rng.choice(T, size=n_pairs, replace=False)
    out = np.zeros((n_pairs, 3), np.int64)
    for j, t in enumerate(traits):
        for _ in range(10000):
            m = int(rng.integers(0, M))
            counts = np.array([(g[m] == c).sum() for c in range(3)])
            if counts.min() >= min_class:
                break
        else:
            raise RuntimeError("no SNP with all three genotype classes")
        model = int(rng.integers(0, 3))
        delta = rng.uniform(0.5, 2.0)
        gm = g[m].astype(np.float64)
        if model == 0:
            eff = gm
        elif model == 1:
            eff = (gm >= 1).astype(np.float64)
        else:
            eff = (gm == int(np.argmin(counts))).astype(np.float64)
        z[t] += delta * eff
        out[j] = (t, m, model)
    return out


def permutations(rng, P, K):
    return np.stack([rng.permutation(K) for _ in range(P)]).astype(np.int32)


# --------------------------------------------------------------------------
# The five workloads (sizes as stated for each).
# --------------------------------------------------------------------------
COHORT_K = (48, 77, 102, 150, 233, 380, 512, 1000)

WORKLOADS = {
    1: dict(name="small_full", K=102, T=1000, M=2000, tie_frac=0.05,
            n_plant=0, p_missing=0.0, P=0, output="full H and p"),
    2: dict(name="paper_scale_hits", K=102, T=20000, M=500000, tie_frac=0.05,
            n_plant=500, p_missing=0.0, P=0, output="hits p<1e-5 + per-trait min p"),
    3: dict(name="precision_K500", K=500, T=20000, M=100000, tie_frac=0.05,
            n_plant=0, p_missing=0.0, P=0, output="three precisions"),
    4: dict(name="permutations", K=102, T=20000, M=100000, tie_frac=0.05,
            n_plant=0, p_missing=0.0, P=200, output="per-perm counts + min p"),
    5: dict(name="cohorts_missing", K=COHORT_K, T=(5000, 20000), M=200000,
            tie_frac=0.05, n_plant=0, p_missing=0.02, P=0, output="hits p<1e-5"),
}


def make_workload(wid, T=None, M=None, K=None, P=None, n_plant=None, seed=None,
                  p_missing=None):
    """Inputs of workload `wid`, optionally resized (T, M, K, P).  Returns a
    dict with expr (T, K) float32, geno (M, K) int8, and when relevant
    planted (n, 3) and perms (P, K) int32."""
    w = dict(WORKLOADS[wid])
    if wid == 5:
        raise ValueError("use make_cohorts for the cohort workload")
    K = K or w["K"]
    T = T or w["T"]
    M = M or w["M"]
    P = w["P"] if P is None else P
    n_plant = w["n_plant"] if n_plant is None else n_plant
    p_missing = w["p_missing"] if p_missing is None else p_missing
    rs = streams(wid if seed is None else seed)
    g, q = genotypes(rs["geno"], M, K)
    g = set_missing(rs["missing"], g, p_missing)
    z = log_normal_z(rs["expr"], T, K)
    planted = plant(rs["plant"], z, g, n_plant) if n_plant else np.zeros((0, 3), np.int64)
    x = inject_ties(rs["ties"], to_expression(z), w["tie_frac"])
    out = dict(expr=x, geno=g, maf=q, planted=planted, K=K, T=T, M=M)
    if P:
        out["perms"] = permutations(rs["perms"], P, K)
    return out


def make_cohorts(M=None, Ks=COHORT_K, T_range=(5000, 20000), T_scale=1.0,
                 p_missing=0.02, seed=5):
    """Cohorts of uneven sample counts sharing one SNP panel: the same SNPs
    (same allele frequencies), each cohort with its own samples.  Returns a
    list of dicts (K, T, expr, geno)."""
    M = M or WORKLOADS[5]["M"]
    rs = streams(seed)
    q = rs["geno"].uniform(0.05, 0.5, size=M)
    out = []
    for c, K in enumerate(Ks):
        T = int(rs["cohort"].integers(T_range[0], T_range[1] + 1))
        T = max(1, int(round(T * T_scale)))
        g, _ = genotypes(rs["geno"], M, K, q=q)
        g = set_missing(rs["missing"], g, p_missing)
        z = log_normal_z(rs["expr"], T, K)
        x = inject_ties(rs["ties"], to_expression(z), 0.05)
        out.append(dict(K=K, T=T, expr=x, geno=g))
    return out
