"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the pin suite against it; the
suite has to fail.  The oracle itself is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "selscan_oracle.c")

MUTANTS = {
    # the term that ends at the first sub-cutoff marker is added
    "adds_stopping_term": (
        """            if (e < p->ehh_cutoff) {
                active[c] = 0;
            } else {
                ihh[c] += 0.5 * (eprev[c] + e) * g;
                eprev[c] = e;
            }""",
        """            ihh[c] += 0.5 * (eprev[c] + e) * g;
            eprev[c] = e;
            if (e < p->ehh_cutoff) active[c] = 0;"""),
    # (">=" instead of ">" on the scaling threshold is not a mistake that can
    #  show: at exactly gap_scale_bp the factor is 1)
    "max_gap_not_strict": ("if (b > p->max_gap_bp) return OR_GAP;", "if (b >= p->max_gap_bp) return OR_GAP;"),
    "gap_factor_inverted": ("g = g * ((double)p->gap_scale_bp / (double)b);",
                            "g = g * ((double)b / (double)p->gap_scale_bp);"),
    "pooled_start_at_one": ("double eprevA = (double)SA / PA, eprevB = (double)SB / PB;",
                            "double eprevA = 1.0, eprevB = 1.0;"),
    "core_not_in_string": ("for (int64_t h = 0; h < pt->n; ++h) pt->lab[h] = row[h] ? 1 : 0;",
                           "for (int64_t h = 0; h < pt->n; ++h) pt->lab[h] = 0;"),
    "no_half_in_trapezoid": ("ihh[c] += 0.5 * (eprev[c] + e) * g;", "ihh[c] += (eprev[c] + e) * g;"),
    "maf_not_strict": ("if (maf < p->maf_cutoff)", "if (maf <= p->maf_cutoff)"),
    "sd_uses_n": ("sqrt(ss / (double)(N - 1))", "sqrt(ss / (double)N)"),
    "edge_not_aborting": ("if (k < 0 || k >= M) return OR_EDGE;\n        double g;\n        if (segment(pos, gpos, k, dir, p, &g)) return OR_GAP;\n        if (tr && tr->len >= tr->cap) { tr->capped = 1; return OR_CAP; }\n        part_refine(pt, H + k * n);",
                          "if (k < 0 || k >= M) return OR_OK;\n        double g;\n        if (segment(pos, gpos, k, dir, p, &g)) return OR_GAP;\n        if (tr && tr->len >= tr->cap) { tr->capped = 1; return OR_CAP; }\n        part_refine(pt, H + k * n);"),
    "upstream_segment_shifted": ("int64_t lo = dir > 0 ? k - 1 : k;", "int64_t lo = k - 1;"),
    "ratio_swapped": ("unstd[j] = log(i1 / i0);", "unstd[j] = log(i0 / i1);"),
    # the upstream abort reported ahead of the downstream one (reading R15)
    "ihs_status_precedence_swapped": (
        "int st = s_dn != OR_OK ? s_dn : s_up;\n            if (st != OR_OK) { status[j] = (int8_t)st; continue; }\n            double i0",
        "int st = s_up != OR_OK ? s_up : s_dn;\n            if (st != OR_OK) { status[j] = (int8_t)st; continue; }\n            double i0"),
    "xpehh_status_precedence_swapped": (
        "int st = s_dn != OR_OK ? s_dn : s_up;\n            if (st != OR_OK) { status[j] = (int8_t)st; continue; }\n            double a =",
        "int st = s_up != OR_OK ? s_up : s_dn;\n            if (st != OR_OK) { status[j] = (int8_t)st; continue; }\n            double a ="),
    # a pooled EHH exactly at the cutoff stops the XPEHH walk (reading R2)
    "pooled_tie_stops": ("if ((double)SP / PP < p->ehh_cutoff) return OR_OK;",
                         "if ((double)SP / PP <= p->ehh_cutoff) return OR_OK;"),
    # the physical-map option ignored, or applied after the gap scaling (R16)
    "physical_map_ignored": ("double g = p->physical_map ? (double)b : gpos[hi] - gpos[lo];",
                             "double g = gpos[hi] - gpos[lo];"),
    "physical_map_unscaled": (
        "    double g = p->physical_map ? (double)b : gpos[hi] - gpos[lo];\n    if (b > p->gap_scale_bp) g = g * ((double)p->gap_scale_bp / (double)b);",
        "    double g = gpos[hi] - gpos[lo];\n    if (b > p->gap_scale_bp) g = g * ((double)p->gap_scale_bp / (double)b);\n    if (p->physical_map) g = (double)b;"),
    "pooled_pairs_across_cores": ("SP += (uint64_t)choose2(pt->cntA[l] + pt->cntB[l]);\n        }\n        if (tr) {\n            tr->len",
                                  "SP += (uint64_t)choose2(pt->cntA[l] + pt->cntB[l]) + (uint64_t)(pt->cntA[l] * pt->cntB[l]);\n        }\n        if (tr) {\n            tr->len"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mutated = src.replace(old, new)
    c = tmp_path / "mutant.c"
    so = tmp_path / "mutant.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    env = dict(os.environ, SS_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutant %s:\n%s" % (name, r.stdout[-2000:])
