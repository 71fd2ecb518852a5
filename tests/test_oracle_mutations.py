"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutation is a plausible slip (a dropped term, an off-by-one, a wrong
sign or index, a swapped distribution); the copy is compiled with gcc and
loaded in place of the real oracle, then the pin battery of
test_oracle_pins is run against it.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "krux_oracle.c")

MUTATIONS = {
    "drop_tie_term": ("int64_t E = Kp * Kp * Kp - Kp - o->tiesum;",
                      "int64_t E = Kp * Kp * Kp - Kp;"),
    "rank_off_by_one": ("a2[k] = (int32_t)(2 * less + eq + 1);",
                        "a2[k] = (int32_t)(2 * less + eq);"),
    "ties_counted_as_less": ("if (x[j] < x[k]) less++;", "if (x[j] <= x[k]) less++;"),
    "wrong_centre": ("int64_t D = o->s2[i] - (int64_t)o->n[i] * (Kp + 1);",
                     "int64_t D = o->s2[i] - (int64_t)o->n[i] * Kp;"),
    "wrong_constant": ("u128 num = (u128)(3 * (Kp - 1)) * P;",
                       "u128 num = (u128)(3 * (Kp + 1)) * P;"),
    "tie_term_t2": ("ts += eq * eq - 1;", "ts += eq - 1;"),
    "df_swapped_tail": ("if (df == 1) return erfc(sqrt(H / 2.0));",
                        "if (df == 1) return exp(-H / 2.0);"),
    "empty_group_not_dropped": ("o->df = nonempty > 0 ? nonempty - 1 : 0;", "o->df = 2;"),
    "missing_not_reranked": ("        rank_row(x, keep, K, a2_tmp, &o->tiesum, &o->kobs);\n        a2 = a2_tmp;",
                             "        (void)a2_tmp;"),
    "rounding_truncates": ("if (round_bit && (sticky || (mant & 1))) mant++;", "(void)sticky;"),
    "threshold_strict": ("if (oracle_pvalue(bitsd(mid), df) >= p_c) lo = mid; else hi = mid;",
                         "if (oracle_pvalue(bitsd(mid), df) > p_c) lo = mid; else hi = mid;"),
    "perm_inverted": ("for (int k = 0; k < K; k++) xp[k] = x[perm[k]];",
                      "for (int k = 0; k < K; k++) xp[perm[k]] = x[k];"),
    "nan_counted_in_group": ("if (gi < 0 || gi > 2 || a2[k] == 0) continue;",
                             "if (gi < 0 || gi > 2) continue;"),
    "genotype_index_shift": ("o->n[gi] += 1;\n        o->s2[gi] += a2[k];",
                             "o->n[gi] += 1;\n        o->s2[(gi + 1) % 3] += a2[k];"),
}

BATTERY = [
    pins.test_worked_examples,
    pins.test_ranks_match_scipy_rankdata,
    pins.test_vs_scipy_kruskal_random,
    pins.test_two_groups_is_mann_whitney_z_squared,
    pins.test_pvalue_matches_chi2_sf,
    pins.test_threshold_is_largest_double_with_p_at_least_pc,
    pins.test_perfect_separation_closed_form,
    pins.test_all_tied_groups_reach_maximum,
    pins.test_degenerate_cases,
    pins.test_invariants,
    pins.test_missing_genotype_equals_kept_samples,
    pins.test_missing_expression_equals_kept_samples,
    pins.test_rational_to_double_matches_fraction,
    pins.test_scan_permutation_is_column_permutation_of_ranks,
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mut = tmp_path / ("krux_oracle_%s.c" % name)
    mut.write_text(src.replace(old, new))
    lib = tmp_path / ("liboracle_%s.so" % name)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-w",
                           "-o", str(lib), str(mut), "-lm"])
    caught = []
    try:
        oracle.use_library(str(lib))
        for t in BATTERY:
            try:
                t()
            except (AssertionError, ValueError, ZeroDivisionError, OverflowError):
                caught.append(t.__name__)
    finally:
        oracle.use_library(None)
    assert caught, "mutation %s passed every pin" % name


# The FDR curve is plain Python in the oracle package: planted mistakes are
# substituted for it directly and must each fail one of its pins.
def _fdr_mutant(name):
    import numpy as np

    def f(real_p, perm_p, P, at=None):
        real_p = np.asarray(real_p, np.float64)
        perm_p = np.asarray(perm_p, np.float64)
        at = real_p if at is None else np.asarray(at, np.float64)
        out = np.empty(len(at))
        for i, q in enumerate(at):
            n_perm = int(np.count_nonzero(perm_p < q if name == "perm_strict" else perm_p <= q))
            n_real = int(np.count_nonzero(real_p < q if name == "real_strict" else real_p <= q))
            if name == "real_total":
                n_real = len(real_p)
            scale = 1.0 if name == "no_mean_over_perms" else float(P)
            out[i] = n_perm / (scale * float(n_real)) if n_real else float("nan")
        return out
    return f


FDR_BATTERY = [pins.test_fdr_curve_worked_example,
               pins.test_fdr_curve_is_mean_of_per_permutation_ratios]


@pytest.mark.parametrize("name", ["perm_strict", "real_strict", "real_total",
                                  "no_mean_over_perms"])
def test_planted_fdr_mistake_is_caught(name, monkeypatch):
    monkeypatch.setattr(oracle, "fdr_curve", _fdr_mutant(name))
    caught = []
    for t in FDR_BATTERY:
        try:
            t()
        except (AssertionError, ValueError, ZeroDivisionError):
            caught.append(t.__name__)
    assert caught, "mutation %s passed every pin" % name
