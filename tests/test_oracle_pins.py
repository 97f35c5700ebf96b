"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests retypes the oracle's formulas: they check it against the
paper's worked example (a golden fixture), brute-force pair enumeration,
closed forms computed exactly with fractions, invariants and symmetries.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from hapgen import random_haplotypes

HERE = os.path.dirname(os.path.abspath(__file__))
P = oracle.Params()
OK, MAF, EDGE, GAP, UNDEF, BIN = 0, 1, 2, 3, 4, 5


def _golden(name):
    out = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


# ---------------------------------------------------------------------------
# Worked example of Sec. 1.1 (golden fixture)
# ---------------------------------------------------------------------------
def test_worked_example_core_and_whole_sample():
    g = _golden("worked_example.txt")
    haps = g["haplotypes"].split()
    H = np.array([[int(h[0]) for h in haps], [int(h[1]) for h in haps]], dtype=np.uint8)
    pos = np.array([1000, 2000], dtype=np.int64)
    gpos = pos * 1e-6
    r = oracle.ehh(H, pos, gpos, core=0, params=P, cap=4, sizes=True)
    # downstream walk reaches x1, EHH stays above the cutoff, then the data end
    assert r["status"] == EDGE
    assert r["len"][0] == 1
    S = r["S"][0]
    assert int(S[0, 1]) == int(g["S1_x0"]) and int(S[0, 0]) == int(g["S0_x0"])
    assert int(S[1, 1]) == int(g["S1_x1"]) and int(S[1, 0]) == int(g["S0_x1"])
    e = r["ehh"][0]
    assert Fraction(e[1, 1]) == Fraction(float(Fraction(g["EHH1_x1"])))
    assert Fraction(e[1, 0]) == Fraction(float(Fraction(g["EHH0_x1"])))
    assert e[0, 2] == float(Fraction(g["EHH_x0"]))
    assert e[1, 2] == float(Fraction(g["EHH_x1"]))
    # classes at x1: four classes of two, two per core (H_1 = {11,10}, H_0 = {00,01})
    sizes = sorted(int(v) for v in r["sizes"][0, 1] if v)
    want = sorted(int(c.split(":")[1]) | ((int(c[0])) << 31) for c in g["classes_x1"].split())
    assert sizes == want
    assert sum(1 for v in r["sizes"][0, 1] if v and (int(v) >> 31) == 1) == len(g["H1_x1"].split())
    assert sum(1 for v in r["sizes"][0, 1] if v and (int(v) >> 31) == 0) == len(g["H0_x1"].split())


def test_worked_example_pooled():
    # The same eight haplotypes split into two populations of four.
    g = _golden("worked_example.txt")
    haps = g["haplotypes"].split()
    H = np.array([[int(h[0]) for h in haps], [int(h[1]) for h in haps]], dtype=np.uint8)
    A = H[:, ::2].copy()   # 11 10 00 01
    B = H[:, 1::2].copy()  # 11 10 00 01
    pos = np.array([1000, 2000], dtype=np.int64)
    r = oracle.xpehh_trace(A, B, pos, pos * 1e-6, site=0, cap=4)
    S = r["S"][0]
    # pooled whole-sample EHH at x0 and x1 (Eq. 1): 12/28 and 4/28
    assert Fraction(int(S[0, 2]), 28) == Fraction(g["EHH_x0"])
    assert Fraction(int(S[1, 2]), 28) == Fraction(g["EHH_x1"])
    # each population alone: two pairs share the core allele at x0, none at x1
    assert int(S[0, 0]) == 2 and int(S[0, 1]) == 2
    assert int(S[1, 0]) == 0 and int(S[1, 1]) == 0


# ---------------------------------------------------------------------------
# Brute-force pair enumeration (integer sums must match exactly)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(60))
def test_core_sums_match_pair_enumeration(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 18))
    M = int(rng.integers(2, 30))
    if seed % 3 == 0:
        d = random_haplotypes(n, M, seed, n_founders=3, switch_p=0.1)
    else:
        d = random_haplotypes(n, M, seed, p=float(rng.uniform(0.2, 0.8)))
    H = d.alleles
    core = int(rng.integers(0, M))
    params = oracle.Params(ehh_cutoff=1e-9)   # walk until every pair has split
    r = oracle.ehh(H, d.pos_bp, d.gpos_cm, core, params, cap=64, sizes=True)
    Hl = H.tolist()
    for di, direction in enumerate((+1, -1)):
        for i in range(int(r["len"][di]) + 1):
            s0, s1 = brute.core_sums(Hl, core, i, direction)
            assert int(r["S"][di, i, 0]) == s0
            assert int(r["S"][di, i, 1]) == s1
            # whole-sample EHH numerator (Eq. 1) is S_0 + S_1
            assert s0 + s1 == brute.identical_pairs(Hl, core, i, direction)
            got = sorted(((int(v) >> 31), int(v) & 0x7FFFFFFF) for v in r["sizes"][di, i] if v)
            assert got == brute.class_sizes(Hl, core, i, direction)


@pytest.mark.parametrize("seed", range(30))
def test_pooled_sums_match_pair_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    nA = int(rng.integers(2, 10))
    nB = int(rng.integers(2, 10))
    M = int(rng.integers(2, 25))
    a = random_haplotypes(nA, M, 200 + seed, p=0.5)
    b = random_haplotypes(nB, M, 300 + seed, p=0.4)
    site = int(rng.integers(0, M))
    r = oracle.xpehh_trace(a.alleles, b.alleles, a.pos_bp, a.gpos_cm, site,
                           oracle.Params(ehh_cutoff=1e-9), cap=64)
    Al, Bl = a.alleles.tolist(), b.alleles.tolist()
    for di, direction in enumerate((+1, -1)):
        for i in range(int(r["len"][di]) + 1):
            sa, sb, sp = brute.pooled_sums(Al, Bl, site, i, direction)
            assert tuple(int(x) for x in r["S"][di, i]) == (sa, sb, sp)


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(10))
def test_ehh_core_starts_at_one_and_never_increases(seed):
    d = random_haplotypes(40, 200, seed, n_founders=5, switch_p=0.02)
    core = 100
    r = oracle.ehh(d.alleles, d.pos_bp, d.gpos_cm, core, P, cap=256)
    n1 = int(d.alleles[core].sum())
    for di in range(2):
        L = int(r["len"][di])
        for c, nc in ((0, 40 - n1), (1, n1)):
            if nc >= 2:
                assert r["ehh"][di, 0, c] == 1.0        # Eq. 3 with one class per core
            s = r["S"][di, : L + 1, c].astype(np.int64)
            assert np.all(np.diff(s) <= 0)             # the partition only refines


def _two_core_block(n_per_core, width, spacing, killer=True):
    """Core site in the middle of 2*width+1 markers; every haplotype is
    identical away from the core, except (if killer) at the outermost markers
    where the two haplotypes of each core differ."""
    M = 2 * width + 1 + (2 if killer else 0)
    n = 2 * n_per_core
    H = np.zeros((M, n), dtype=np.uint8)
    core = M // 2
    H[core, :n_per_core] = 1
    if killer:
        for s in (0, M - 1):
            H[s, 0] = 1              # splits core 1's pair
            H[s, n_per_core] = 1     # splits core 0's pair
    pos = (np.arange(M, dtype=np.int64) + 1) * spacing
    gpos = np.arange(M, dtype=np.float64) * 0.0625   # dyadic: differences are exact
    return H, pos, gpos, core


def test_identical_haplotypes_reach_the_edge_with_ehh_one():
    H, pos, gpos, core = _two_core_block(5, 20, 1000, killer=False)
    r = oracle.ehh(H, pos, gpos, core, P, cap=64)
    assert r["status"] == EDGE
    for di in range(2):
        L = int(r["len"][di])
        assert L == 20
        assert np.all(r["ehh"][di, : L + 1, :2] == 1.0)
    out = oracle.ihs(H, pos, gpos, P)
    assert out["status"][core] == EDGE


@pytest.mark.parametrize("spacing,scale", [(10_000, Fraction(1)), (20_000, Fraction(1)),
                                           (40_000, Fraction(1, 2))])
def test_constant_curve_integrates_to_total_scaled_distance(spacing, scale):
    # EHH_c = 1 on the whole window, then 0 at the killer markers: the killer
    # step adds no term (truncation reading), so iHH = total scaled distance.
    w = 7
    H, pos, gpos, core = _two_core_block(2, w, spacing, killer=True)
    out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0))
    assert out["status"][core] in (OK, BIN)
    want = Fraction(2 * w) * Fraction(0.0625) * scale
    assert Fraction(out["ihh1"][core]) == want
    assert Fraction(out["ihh0"][core]) == want
    assert out["unstd"][core] == 0.0
    assert out["steps"][core].tolist() == [[w + 1, w + 1], [w + 1, w + 1]]


def test_gap_thresholds_are_strict():
    w = 4
    for spacing, status in ((200_000, (OK, BIN)), (200_001, (GAP,))):
        H, pos, gpos, core = _two_core_block(2, w, spacing, killer=True)
        out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0))
        assert out["status"][core] in status, (spacing, out["status"][core])


def test_gap_on_the_stopping_segment_aborts():
    # The walk would stop at the killer marker, but the segment leading to it
    # is longer than the abort gap: the locus is aborted.
    w = 4
    H, pos, gpos, core = _two_core_block(2, w, 1000, killer=True)
    pos = pos.copy()
    pos[-1] = pos[-2] + 250_000
    out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0))
    assert out["status"][core] == GAP


def test_gap_beyond_the_stop_is_ignored():
    w = 4
    H, pos, gpos, core = _two_core_block(2, w, 1000, killer=True)
    H = np.vstack([H, np.zeros((1, H.shape[1]), dtype=np.uint8)])
    pos = np.append(pos, pos[-1] + 500_000)
    gpos = np.append(gpos, gpos[-1] + 0.0625)
    out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0))
    assert out["status"][core] in (OK, BIN)


def _peel(k1, k0, spacing, gstep):
    """One haplotype of each core leaves its class at every marker on either
    side of the core, so S_c(i) = C(k_c - i, 2) in both directions."""
    K = max(k1, k0)
    M = 2 * K + 1
    n = k1 + k0
    H = np.zeros((M, n), dtype=np.uint8)
    core = K
    H[core, :k1] = 1
    for i in range(1, K + 1):
        for s in (core + i, core - i):
            if i - 1 < k1:
                H[s, i - 1] = 1
            if i - 1 < k0:
                H[s, k1 + i - 1] = 1
    pos = (np.arange(M, dtype=np.int64) + 1) * spacing
    gpos = np.arange(M, dtype=np.float64) * gstep
    return H, pos, gpos, core


def _peel_ihh_exact(k, cutoff, g):
    """Exact trapezoid of EHH(i) = C(k-i,2)/C(k,2) with step g, truncated
    before the first i with EHH(i) < cutoff; one direction."""
    P = Fraction(k * (k - 1), 2)
    total = Fraction(0)
    prev = Fraction(1)
    i = 0
    while True:
        i += 1
        e = Fraction((k - i) * (k - i - 1), 2) / P if k - i >= 2 else Fraction(0)
        # the cutoff test compares the correctly rounded ratio with the cutoff;
        # k = 25 hits EHH = 15/300 = 1/20 exactly, which rounds to the double
        # 0.05 and so does not stop the walk
        if float(e) < cutoff:
            return total, i
        total += (prev + e) / 2 * g
        prev = e


@pytest.mark.parametrize("k1,k0,spacing", [(12, 9, 10_000), (30, 17, 5_000), (25, 40, 30_000)])
def test_peel_construction_closed_form(k1, k0, spacing):
    gstep = 0.0625
    H, pos, gpos, core = _peel(k1, k0, spacing, gstep)
    out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0))
    assert out["status"][core] in (OK, BIN)
    g = Fraction(gstep)
    if spacing > 20_000:
        g = g * Fraction(20_000, spacing)
    exact = {}
    for c, k in ((1, k1), (0, k0)):
        one_side, stop = _peel_ihh_exact(k, 0.05, g)
        want = 2 * one_side
        exact[c] = want
        got = out["ihh1" if c else "ihh0"][core]
        assert abs(Fraction(got) - want) <= Fraction(1, 10**15) * want
        assert out["steps"][core, 0, c] == stop and out["steps"][core, 1, c] == stop
    # Eq. 5 orientation: ln(iHH_1 / iHH_0), positive when the derived core's
    # haplotypes extend further
    u = out["unstd"][core]
    assert abs(u - math.log(exact[1] / exact[0])) <= 1e-14 * max(1.0, abs(u))
    assert (u > 0) == (exact[1] > exact[0])


def test_xpehh_constant_curves_closed_form():
    # A: 4 derived + 2 ancestral, B: 3 + 3, identical away from the core.
    # Whole-sample EHH at x0 (Eq. 1, x0 part of the string): A 7/15, B 6/15.
    # The outermost markers split the pooled sample by population only, so
    # each population's EHH stays constant while the pooled EHH falls from
    # 31/66 to 13/66, below the cutoff 0.25: both walks stop there, without
    # a term, and iHH_X = EHH_X(x0) * (total scaled distance).
    w = 6
    M = 2 * w + 3
    A = np.zeros((M, 6), dtype=np.uint8)
    B = np.zeros((M, 6), dtype=np.uint8)
    core = M // 2
    A[core, :4] = 1
    B[core, :3] = 1
    B[0, :] = 1
    B[M - 1, :] = 1
    pos = (np.arange(M, dtype=np.int64) + 1) * 30_000
    gpos = np.arange(M, dtype=np.float64) * 0.0625
    out = oracle.xpehh(A, B, pos, gpos, oracle.Params(ehh_cutoff=0.25))
    D = Fraction(2 * w) * Fraction(0.0625) * Fraction(20_000, 30_000)
    ia, ib = Fraction(7, 15) * D, Fraction(6, 15) * D
    assert abs(Fraction(out["ihhA"][core]) - ia) <= Fraction(1, 10**15) * ia
    assert abs(Fraction(out["ihhB"][core]) - ib) <= Fraction(1, 10**15) * ib
    assert abs(out["unstd"][core] - math.log(7 / 6)) <= 1e-15
    assert out["steps"][core].tolist() == [w + 1, w + 1]


# ---------------------------------------------------------------------------
# Symmetries
# ---------------------------------------------------------------------------
def _dyadic(M, seed):
    """Uneven spacing with dyadic genetic positions, so that differences of
    genetic positions are exact and mirroring changes no segment length."""
    d = random_haplotypes(60, M, seed, n_founders=6, switch_p=0.03)
    rng = np.random.default_rng(seed + 1000)
    pos = np.cumsum(rng.integers(300, 30_000, size=M)).astype(np.int64)
    gpos = np.cumsum(rng.integers(1, 64, size=M)).astype(np.float64) / 1024.0
    return d.alleles, pos, gpos


def test_haplotype_permutation_is_bit_exact():
    H, pos, gpos = _dyadic(300, 5)
    a = oracle.ihs(H, pos, gpos, P)
    perm = np.random.default_rng(1).permutation(H.shape[1])
    b = oracle.ihs(H[:, perm], pos, gpos, P)
    for k in ("ihh1", "ihh0", "unstd", "std"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(a["status"], b["status"])


def test_allele_flips_away_from_the_core_and_core_swap():
    H, pos, gpos = _dyadic(300, 6)
    base = oracle.ihs(H, pos, gpos, P)
    loci = np.nonzero(base["status"] == OK)[0][:40]
    assert len(loci) > 10
    for j in loci:
        F = H ^ 1
        F[j] = H[j]                      # flip every marker but the core
        r = oracle.ihs(F, pos, gpos, P, loci=[j])
        assert r["ihh1"][j] == base["ihh1"][j] and r["ihh0"][j] == base["ihh0"][j]
        G = H.copy()
        G[j] ^= 1                        # swap the core labels
        s = oracle.ihs(G, pos, gpos, P, loci=[j])
        assert s["ihh1"][j] == base["ihh0"][j] and s["ihh0"][j] == base["ihh1"][j]
        assert abs(s["unstd"][j] + base["unstd"][j]) <= 1e-15 * max(1.0, abs(base["unstd"][j]))


def test_mirrored_marker_order_is_bit_exact():
    H, pos, gpos = _dyadic(300, 7)
    M = H.shape[0]
    a = oracle.ihs(H, pos, gpos, P)
    Hm = H[::-1].copy()
    posm = (pos[-1] + pos[0]) - pos[::-1]
    gposm = (gpos[-1] + gpos[0]) - gpos[::-1]
    b = oracle.ihs(Hm, posm, gposm, P)
    np.testing.assert_array_equal(a["ihh1"], b["ihh1"][::-1])
    np.testing.assert_array_equal(a["ihh0"], b["ihh0"][::-1])
    np.testing.assert_array_equal(a["status"], b["status"][::-1])
    assert M == Hm.shape[0]


def test_xpehh_against_itself_is_zero_and_antisymmetric():
    a = random_haplotypes(30, 250, 11, n_founders=5, switch_p=0.03)
    b = random_haplotypes(26, 250, 12, n_founders=4, switch_p=0.02)
    self_ = oracle.xpehh(a.alleles, a.alleles, a.pos_bp, a.gpos_cm, P)
    # every u is 0, so the genome-wide SD is 0 and the scores land in BIN
    ok = (self_["status"] == OK) | (self_["status"] == BIN)
    assert ok.sum() > 50
    assert np.all(self_["unstd"][ok] == 0.0)
    assert np.all(self_["ihhA"][ok] == self_["ihhB"][ok])
    ab = oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm, P)
    ba = oracle.xpehh(b.alleles, a.alleles, a.pos_bp, a.gpos_cm, P)
    np.testing.assert_array_equal(ab["ihhA"], ba["ihhB"])
    np.testing.assert_array_equal(ab["ihhB"], ba["ihhA"])
    m = ab["status"] == OK
    assert np.all(np.abs(ab["unstd"][m] + ba["unstd"][m]) <= 1e-15 * np.maximum(1, np.abs(ab["unstd"][m])))


# ---------------------------------------------------------------------------
# MAF filter, bins and standardization
# ---------------------------------------------------------------------------
def test_maf_filter_is_strict_and_bins_are_integer():
    n = 40
    M = 41
    H = np.zeros((M, n), dtype=np.uint8)
    for j in range(M):
        H[j, :j] = 1                      # n1 = j at site j (n1 = 40 at the last site)
    pos = (np.arange(M, dtype=np.int64) + 1) * 1000
    out = oracle.ihs(H, pos, pos * 1e-6, P)
    for j in range(M):
        maf = min(j, n - j) / n
        assert (out["status"][j] == MAF) == (maf < 0.05)
        assert out["bin"][j] == min(40 * j // n, 39)
        assert out["freq"][j] == j / n
    assert out["status"][2] != MAF       # MAF exactly 0.05 is scored


def test_standardization_matches_numpy_per_bin():
    from hapgen import config_input
    d = config_input(0)
    out = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, P)
    ok = (out["status"] == OK)
    assert ok.sum() > 500
    for b in np.unique(out["bin"][ok]):
        m = ok & (out["bin"] == b)
        u = out["unstd"][m]
        z = (u - np.mean(u)) / np.std(u, ddof=1)
        np.testing.assert_allclose(out["std"][m], z, rtol=1e-12, atol=1e-12)
        assert abs(np.mean(out["std"][m])) < 1e-10
        assert abs(np.std(out["std"][m], ddof=1) - 1.0) < 1e-10


def test_undefined_when_a_core_is_too_small():
    n, M = 10, 30
    H = np.zeros((M, n), dtype=np.uint8)
    H[15, 0] = 1                          # one derived copy: C(1,2) = 0
    pos = (np.arange(M, dtype=np.int64) + 1) * 1000
    out = oracle.ihs(H, pos, pos * 1e-6, oracle.Params(maf_cutoff=0.0))
    assert out["status"][15] == UNDEF


def test_last_site_is_an_edge():
    d = random_haplotypes(30, 50, 3, p=0.5)
    out = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, oracle.Params(maf_cutoff=0.0))
    assert out["status"][0] in (EDGE, UNDEF, MAF)
    assert out["status"][-1] in (EDGE, UNDEF, MAF)


# ---------------------------------------------------------------------------
# Which abort a locus reports when its two directions abort differently
# (reading R15: the downstream abort if there is one, else the upstream one)
# ---------------------------------------------------------------------------
def _gap_one_side_edge_other(gap_side, n_per_core=3, w=6):
    """Haplotypes identical away from the core, so every walk stays at
    EHH = 1: on one side a gap longer than the abort gap is crossed two
    markers out, on the other side the walk runs into the end of the data."""
    H, pos, gpos, core = _two_core_block(n_per_core, w, 1000, killer=False)
    pos = pos.copy()
    if gap_side > 0:
        pos[core + 3:] += 250_000          # segment (core+2, core+3) is 251 kb
    else:
        pos[: core - 2] -= 250_000         # segment (core-3, core-2) is 251 kb
    return H, pos, gpos, core


@pytest.mark.parametrize("gap_side,want", [(+1, GAP), (-1, EDGE)])
def test_ihs_status_when_directions_abort_differently(gap_side, want):
    H, pos, gpos, core = _gap_one_side_edge_other(gap_side)
    out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0))
    assert out["status"][core] == want
    assert np.isnan(out["ihh1"][core]) and np.isnan(out["unstd"][core])
    # each direction alone: the gap side gives GAP, the other side EDGE
    r = oracle.ehh(H, pos, gpos, core, P, cap=64)
    assert r["status"] == want


@pytest.mark.parametrize("gap_side,want", [(+1, GAP), (-1, EDGE)])
def test_xpehh_status_when_directions_abort_differently(gap_side, want):
    H, pos, gpos, core = _gap_one_side_edge_other(gap_side)
    A, B = H[:, :4].copy(), H[:, 2:].copy()     # 3+1 and 1+3 derived at the core
    out = oracle.xpehh(A, B, pos, gpos, P)
    assert out["status"][core] == want
    assert np.isnan(out["ihhA"][core]) and np.isnan(out["unstd"][core])


# ---------------------------------------------------------------------------
# Pooled truncation of XPEHH at an exact tie (Sec. 1.3 with reading R2)
# ---------------------------------------------------------------------------
def _pooled_peel(nA, nB):
    """Every pooled haplotype carries the ancestral allele at the core; at
    the i-th marker on either side, haplotype i-1 of the pooled order (A's
    then B's, interleaved) alone carries the derived allele, so it leaves the
    one class: S_pool(i) = C(n - i, 2)."""
    n = nA + nB
    M = 2 * n + 1
    core = n
    order = []                                   # alternate A and B haplotypes
    ia, ib = 0, 0
    while ia < nA or ib < nB:
        if ia < nA:
            order.append(("A", ia)); ia += 1
        if ib < nB:
            order.append(("B", ib)); ib += 1
    A = np.zeros((M, nA), dtype=np.uint8)
    B = np.zeros((M, nB), dtype=np.uint8)
    for i in range(1, n + 1):
        pop, h = order[i - 1]
        for s in (core + i, core - i):
            (A if pop == "A" else B)[s, h] = 1
    pos = (np.arange(M, dtype=np.int64) + 1) * 10_000
    gpos = np.arange(M, dtype=np.float64) * 0.0625
    return A, B, pos, gpos, core, order


def _pooled_peel_exact(nA, nB, order, cutoff, g):
    """One direction, exactly: the pooled stop at the first i with
    fl(S_pool(i)/C(n,2)) < cutoff, each population's trapezoid up to there."""
    n = nA + nB
    PP = Fraction(n * (n - 1), 2)
    left = {"A": nA, "B": nB}
    c2 = lambda k: Fraction(k * (k - 1), 2)
    prev = {"A": Fraction(1), "B": Fraction(1)}
    tot = {"A": Fraction(0), "B": Fraction(0)}
    i = 0
    while True:
        i += 1
        left[order[i - 1][0]] -= 1
        sp = c2(n - i)
        if float(sp / PP) < cutoff:
            return tot, i
        for q, nq in (("A", nA), ("B", nB)):
            e = c2(left[q]) / c2(nq)
            tot[q] += (prev[q] + e) / 2 * g
            prev[q] = e


def test_xpehh_pooled_cutoff_tie_does_not_stop():
    # pooled n = 25: S_pool = C(6, 2) = 15 of C(25, 2) = 300 is exactly 1/20,
    # which rounds to the double 0.05 and so does not stop the walk; the stop
    # comes one marker later at 10/300
    nA, nB = 13, 12
    A, B, pos, gpos, core, order = _pooled_peel(nA, nB)
    out = oracle.xpehh(A, B, pos, gpos, P)
    tot, stop = _pooled_peel_exact(nA, nB, order, 0.05, Fraction(0.0625))
    assert stop == 20
    assert out["steps"][core].tolist() == [stop, stop]
    for q, key in (("A", "ihhA"), ("B", "ihhB")):
        want = 2 * tot[q]
        assert abs(Fraction(out[key][core]) - want) <= Fraction(1, 10**15) * want
    tr = oracle.xpehh_trace(A, B, pos, gpos, core, P, cap=64)
    assert int(tr["S"][0, 19, 2]) == 15 and int(tr["S"][0, 20, 2]) == 10


# ---------------------------------------------------------------------------
# Physical-map option (reading R16): g = physical distance in bp, gap rules
# unchanged
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("spacing,seg_bp", [(10_000, 10_000), (20_000, 20_000), (40_000, 20_000),
                                            (160_000, 20_000)])
def test_physical_map_constant_curve_closed_form(spacing, seg_bp):
    # EHH = 1 over the window: iHH is the total scaled physical distance; a
    # gap above 20 kb counts 20,000 bp (g = b * 20000 / b)
    w = 5
    H, pos, gpos, core = _two_core_block(2, w, spacing, killer=True)
    out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0, physical_map=1))
    assert out["status"][core] in (OK, BIN)
    assert out["ihh1"][core] == 2 * w * seg_bp
    assert out["ihh0"][core] == 2 * w * seg_bp


def test_physical_map_peel_closed_form():
    H, pos, gpos, core = _peel(14, 11, 7_000, 0.0625)
    out = oracle.ihs(H, pos, gpos, oracle.Params(maf_cutoff=0.0, physical_map=1))
    for c, k in ((1, 14), (0, 11)):
        one_side, stop = _peel_ihh_exact(k, 0.05, Fraction(7_000))
        got = out["ihh1" if c else "ihh0"][core]
        assert abs(Fraction(got) - 2 * one_side) <= Fraction(1, 10**15) * 2 * one_side
        assert out["steps"][core, 0, c] == stop


@pytest.mark.parametrize("kind", ["ihs", "xpehh"])
def test_physical_map_equals_a_constant_rate_genetic_map(kind):
    # gpos = pos * 2^-20: every genetic segment is the physical one times a
    # power of two, so every iHH scales by it exactly and the scores agree
    # bit for bit (gaps above 20 kb and above 200 kb included)
    d = random_haplotypes(80, 600, 17, n_founders=8, switch_p=0.02)
    rng = np.random.default_rng(5)
    steps = rng.integers(200, 9_000, size=600)
    steps[rng.choice(600, 20, replace=False)] = rng.integers(20_001, 60_000, 20)
    steps[rng.choice(600, 3, replace=False)] = 250_000
    pos = np.cumsum(steps).astype(np.int64)
    r = 2.0 ** -20
    gpos = pos.astype(np.float64) * r
    phys = oracle.Params(physical_map=1)
    if kind == "ihs":
        g = oracle.ihs(d.alleles, pos, gpos, P)
        p = oracle.ihs(d.alleles, pos, gpos, phys)
        keys = ("ihh1", "ihh0")
    else:
        e = random_haplotypes(70, 600, 18, n_founders=8, switch_p=0.02)
        g = oracle.xpehh(d.alleles, e.alleles, pos, gpos, P)
        p = oracle.xpehh(d.alleles, e.alleles, pos, gpos, phys)
        keys = ("ihhA", "ihhB")
    np.testing.assert_array_equal(g["status"], p["status"])
    assert (g["status"] == OK).sum() > 100 and (g["status"] == GAP).sum() > 0
    for k in keys:
        np.testing.assert_array_equal(g[k], p[k] * r)
    np.testing.assert_array_equal(g["unstd"], p["unstd"])
    np.testing.assert_array_equal(g["std"], p["std"])


# ---------------------------------------------------------------------------
# Genome-wide standardization over several scans (Eq. 6 and Eq. 9 across the
# entire genome)
# ---------------------------------------------------------------------------
def _scans_for_genome():
    outs = []
    for n, m, seed in ((90, 700, 31), (150, 900, 32), (40, 300, 33)):
        d = random_haplotypes(n, m, seed, n_founders=max(3, n // 12), switch_p=0.02)
        outs.append(oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, P))
    return outs


def test_genome_standardization_matches_numpy_over_the_concatenation():
    outs = _scans_for_genome()
    res, stats = oracle.genome_standardize(outs, 40)
    u = np.concatenate([o["unstd"] for o in outs])
    scored = np.isin(np.concatenate([o["status"] for o in outs]), (OK, BIN))
    bins = np.concatenate([o["bin"] for o in outs])
    z = np.concatenate([r["std"] for r in res])
    st = np.concatenate([r["status"] for r in res])
    checked = 0
    for b in range(40):
        m = scored & (bins == b)
        assert stats["n"][b] == m.sum()
        if m.sum() < 2:
            assert np.all(st[m] == BIN) and np.all(np.isnan(z[m]))
            continue
        v = u[m]
        np.testing.assert_allclose(z[m], (v - v.mean()) / v.std(ddof=1), rtol=1e-12, atol=1e-12)
        assert np.all(st[m] == OK)
        checked += 1
    assert checked > 10
    assert np.all(np.isnan(z[~scored])) and np.array_equal(st[~scored],
                                                          np.concatenate([o["status"] for o in outs])[~scored])


@pytest.mark.parametrize("kind", ["ihs", "xpehh"])
def test_genome_standardization_of_pieces_equals_the_whole(kind):
    # one scan's scores cut into pieces, each standardized on its own (small
    # pieces leave bins with fewer than 2 loci: status BIN), then standardized
    # together, give exactly the standardization of the whole scan
    d = random_haplotypes(120, 1500, 41, n_founders=10, switch_p=0.02)
    if kind == "ihs":
        whole = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, P)
        nbins = 40
    else:
        e = random_haplotypes(100, 1500, 42, n_founders=9, switch_p=0.02)
        whole = oracle.xpehh(d.alleles, e.alleles, d.pos_bp, d.gpos_cm, P)
        whole["bin"] = np.zeros(1500, dtype=np.int32)
        nbins = 1
    pre = np.where(whole["status"] == BIN, OK, whole["status"]).astype(np.int8)
    k = int(np.flatnonzero(pre[600:] == OK)[0]) + 600     # a one-locus piece: BIN on its own
    pieces = []
    for a, b in ((0, 37), (37, 600), (600, k), (k, k + 1), (k + 1, 1500)):
        r = oracle.standardize(whole["unstd"][a:b], pre[a:b], whole["bin"][a:b], nbins)
        pieces.append({"unstd": whole["unstd"][a:b], "status": r["status"], "bin": whole["bin"][a:b]})
    assert any((p["status"] == BIN).any() for p in pieces)
    res, _ = oracle.genome_standardize(pieces, nbins)
    np.testing.assert_array_equal(np.concatenate([r["std"] for r in res]), whole["std"])
    np.testing.assert_array_equal(np.concatenate([r["status"] for r in res]), whole["status"])
