"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Bars: integer results (class sums S, class sizes, walk lengths, per-site
status and steps) bit-exact; EHH and iHH within 1e-12 relative; log-ratios
and standardized scores within 1e-12 * max(|a|, |b|, 1), because a log-ratio
near 0 has no useful pure-relative bound unless both sides use the same libm.
"""
import sys
import zlib

import numpy as np
import pytest

import hapgen
import oracle
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

REL = 1e-12


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ss():
    import paper_1403_6854_amd as ss
    ss.lib()
    return ss


@pytest.fixture(params=[1, 2, "batch_ids", "batch_lists"],
                ids=["lds_ids", "reg_masks", "batch_ids", "batch_lists"])
def walk(request, ss):
    """Run a scan test with each EHH-walk kernel (results must not depend on
    it): the plain class-id kernel, the bitmask kernel, and both kernels of the
    persistent batch walk."""
    if request.param == "batch_ids":
        ss.set_batch_config(ss.BatchConfig(kernel=0))
        ss.set_walk_kernel(3)
    elif request.param == "batch_lists":
        ss.set_batch_config(ss.BatchConfig(kernel=1, threads=256))
        ss.set_walk_kernel(3)
    else:
        ss.set_walk_kernel(request.param)
    yield request.param
    ss.set_walk_kernel(0)
    ss.set_batch_config(ss.BatchConfig())


def _dev(d):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(d.alleles)).cuda(),
            torch.from_numpy(d.pos_bp).cuda(), torch.from_numpy(d.gpos_cm).cuda())


def _hm(ss, alleles, pos, gpos):
    import torch
    return ss.hapmat(torch.from_numpy(np.ascontiguousarray(alleles)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(pos, dtype=np.int64)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(gpos, dtype=np.float64)).cuda())


def _np(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def assert_rel(a, b, mask, what):
    a, b = a[mask], b[mask]
    assert np.array_equal(np.isnan(a), np.isnan(b)), what + ": NaN pattern differs"
    f = ~np.isnan(a)
    err = np.abs(a[f] - b[f])
    lim = REL * np.maximum(np.abs(a[f]), np.abs(b[f]))
    assert np.all(err <= lim), "%s: max rel err %.3g" % (
        what, float(np.max(err / np.maximum(lim / REL, 1e-300))) if err.size else 0.0)


def assert_log(a, b, mask, what):
    a, b = a[mask], b[mask]
    assert np.array_equal(np.isnan(a), np.isnan(b)), what + ": NaN pattern differs"
    f = ~np.isnan(a)
    err = np.abs(a[f] - b[f])
    lim = REL * np.maximum(1.0, np.maximum(np.abs(a[f]), np.abs(b[f])))
    assert np.all(err <= lim), "%s: max err %.3g" % (what, float(err.max()) if err.size else 0.0)


def check_ihs(got, ref, what):
    assert np.array_equal(got["status"], ref["status"]), what + ": status"
    assert np.array_equal(got["steps"], ref["steps"].astype(np.int32)), what + ": steps"
    np.testing.assert_array_equal(got["freq"], ref["freq"])
    every = np.ones(len(ref["status"]), dtype=bool)
    assert_rel(got["ihh1"], ref["ihh1"], every, what + ": ihh1")
    assert_rel(got["ihh0"], ref["ihh0"], every, what + ": ihh0")
    assert_log(got["unstd"], ref["unstd"], every, what + ": unstd")
    assert_log(got["std"], ref["std"], every, what + ": std")


def check_xpehh(got, ref, what):
    assert np.array_equal(got["status"], ref["status"]), what + ": status"
    assert np.array_equal(got["steps"], ref["steps"].astype(np.int32)), what + ": steps"
    every = np.ones(len(ref["status"]), dtype=bool)
    assert_rel(got["ihhA"], ref["ihhA"], every, what + ": ihhA")
    assert_rel(got["ihhB"], ref["ihhB"], every, what + ": ihhB")
    assert_log(got["unstd"], ref["unstd"], every, what + ": unstd")
    assert_log(got["std"], ref["std"], every, what + ": std")


# ---------------------------------------------------------------------------
# ss_ehh: per-marker integer sums and class sizes, bit-exact
# ---------------------------------------------------------------------------
def _ehh_case(ss, d, core, params=oracle.Params(), cap=2048):
    say("ss_ehh n=%d M=%d core=%d cutoff=%g" % (d.n_haps, d.n_sites, core, params.ehh_cutoff))
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    got = _np(ss.ehh(h, core, ss.Params(**vars(params)), cap=cap, sizes=True))
    ref = oracle.ehh(d.alleles, d.pos_bp, d.gpos_cm, core, params, cap=cap, sizes=True)
    assert int(got["status"][0]) == ref["status"], "status"
    np.testing.assert_array_equal(got["len"], ref["len"])
    for di in range(2):
        L = int(ref["len"][di])
        np.testing.assert_array_equal(got["S"][di, : L + 1].astype(np.uint64), ref["S"][di, : L + 1])
        e_g, e_r = got["ehh"][di, : L + 1], ref["ehh"][di, : L + 1]
        assert np.array_equal(np.isnan(e_g), np.isnan(e_r))
        np.testing.assert_array_equal(e_g[~np.isnan(e_g)], e_r[~np.isnan(e_r)])
        for i in range(L + 1):
            a = np.sort(got["sizes"][di, i].view(np.uint32))
            b = np.sort(ref["sizes"][di, i])
            np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(np.isnan(got["ihh"]), np.isnan(ref["ihh"]))
    f = ~np.isnan(ref["ihh"])
    assert np.all(np.abs(got["ihh"][f] - ref["ihh"][f]) <= REL * np.abs(ref["ihh"][f]))


def test_ehh_worked_example_shapes(ss):
    d = hapgen.config_input(0)
    for core in (0, 1, 57, 999, 1500, 1998, 1999):
        _ehh_case(ss, d, core)


@pytest.mark.parametrize("n", [2, 3, 5, 63, 64, 65, 127, 128, 129, 300, 700])
def test_ehh_ragged_haplotype_counts(ss, n):
    d = hapgen.random_haplotypes(n, 400, 10 + n, n_founders=max(2, n // 10), switch_p=0.02)
    for core in (0, 133, 399):
        _ehh_case(ss, d, core, oracle.Params(ehh_cutoff=0.01), cap=512)


def test_ehh_long_sweep_walk(ss):
    d = hapgen.config_input(1)
    j = d.sweep_sites[0]
    for core in (j, j - 40, j + 100):
        _ehh_case(ss, d, core, cap=4096)


def test_ehh_capacity_status(ss):
    d = hapgen.config_input(1)
    j = d.sweep_sites[0]
    say("ss_ehh capacity case")
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    got = _np(ss.ehh(h, j, cap=8))
    ref = oracle.ehh(d.alleles, d.pos_bp, d.gpos_cm, j, cap=8)
    assert int(got["status"][0]) == ref["status"] == 6
    np.testing.assert_array_equal(got["len"], ref["len"])


# ---------------------------------------------------------------------------
# ss_ihs
# ---------------------------------------------------------------------------
def test_ihs_tiny_config(ss, walk):
    d = hapgen.config_input(0)
    say("ss_ihs 200 x 2000 walk=%s" % walk)
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    got = _np(ss.ihs(h, steps=True))
    ref = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm)
    check_ihs(got, ref, "tiny")


def test_ihs_chr22_shaped_config(ss, walk):
    d = hapgen.config_input(1)
    say("ss_ihs 204 x 22147 walk=%s" % walk)
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    got = _np(ss.ihs(h, steps=True))
    ref = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm)
    check_ihs(got, ref, "chr22")
    assert (ref["status"] == 0).sum() > 10000


@pytest.mark.parametrize("case", ["gaps", "dup_positions", "maf0", "cutoff_high", "cutoff_low",
                                  "narrow_bins", "one_site", "two_haps"])
def test_ihs_edge_cases(ss, walk, case):
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    params = oracle.Params()
    if case == "one_site":
        d = hapgen.random_haplotypes(20, 1, 1)
    elif case == "two_haps":
        d = hapgen.random_haplotypes(2, 300, 2)
        params = oracle.Params(maf_cutoff=0.0)
    else:
        d = hapgen.random_haplotypes(150, 1500, 3, n_founders=12, switch_p=0.01)
    pos = d.pos_bp.copy()
    if case == "gaps":
        steps = rng.integers(1000, 6000, size=len(pos))
        steps[rng.choice(len(pos), 12, replace=False)] = 25_000 + rng.integers(0, 10_000, 12)
        steps[rng.choice(len(pos), 4, replace=False)] = 250_000
        steps[100] = 200_000
        steps[700] = 200_001
        steps[900] = 20_000
        steps[901] = 20_001
        pos = np.cumsum(steps).astype(np.int64)
    if case == "dup_positions":
        pos = np.repeat(np.arange(len(pos) // 2 + 1) * 2000, 2)[: len(pos)].astype(np.int64) + 1
    gpos = pos * 1e-6
    if case == "maf0":
        params = oracle.Params(maf_cutoff=0.0)
    if case == "cutoff_high":
        params = oracle.Params(ehh_cutoff=0.5)
    if case == "cutoff_low":
        params = oracle.Params(ehh_cutoff=0.001)
    if case == "narrow_bins":
        params = oracle.Params(bin_width=0.01)
    say("ss_ihs edge case %s walk=%s" % (case, walk))
    h = _hm(ss, d.alleles, pos, gpos)
    got = _np(ss.ihs(h, ss.Params(**vars(params)), steps=True))
    ref = oracle.ihs(d.alleles, pos, gpos, params)
    check_ihs(got, ref, case)


@pytest.mark.parametrize("n", [3, 63, 64, 65, 128, 129, 256, 257, 400, 511, 512, 513, 700, 1024, 1025])
def test_ihs_ragged_haplotype_counts(ss, walk, n):
    d = hapgen.random_haplotypes(n, 700, 40 + n, n_founders=max(2, n // 12), switch_p=0.01)
    say("ss_ihs %d x 700 walk=%s" % (n, walk))
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    params = oracle.Params(maf_cutoff=0.0)
    got = _np(ss.ihs(h, ss.Params(**vars(params)), steps=True))
    ref = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, params)
    check_ihs(got, ref, "n=%d" % n)


@pytest.mark.parametrize("lpc,n", [(lpc, n) for lpc in (1, 2, 4, 8) for n in (65, 204, 300, 510)]
                         + [(2, 700), (4, 700), (2, 1000), (4, 1000)])
def test_ihs_mask_lanes(ss, lpc, n):
    # every lanes-per-class setting of the bitmask walk gives the same answer
    d = hapgen.random_haplotypes(n, 900, 70 + n, n_founders=max(2, n // 10), switch_p=0.006)
    say("ss_ihs %d x 900 mask lanes=%d" % (n, lpc))
    ss.set_walk_kernel(2)
    ss.set_mask_lanes(lpc)
    try:
        h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
        got = _np(ss.ihs(h, steps=True))
    finally:
        ss.set_mask_lanes(0)
        ss.set_walk_kernel(0)
    ref = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm)
    check_ihs(got, ref, "n=%d lpc=%d" % (n, lpc))


@pytest.mark.parametrize("lpc,na,nb", [(lpc, 200, 190) for lpc in (1, 2, 4, 8)] + [(2, 420, 380), (4, 420, 380)])
def test_xpehh_mask_lanes(ss, lpc, na, nb):
    # 200 + 190: 8-word pooled masks; 420 + 380: 16-word masks, 2 or 4 lanes a class
    a = hapgen.random_haplotypes(na, 800, 5, n_founders=15, switch_p=0.004)
    b = hapgen.random_haplotypes(nb, 800, 6, n_founders=12, switch_p=0.004)
    say("ss_xpehh %d+%d x 800 mask lanes=%d" % (na, nb, lpc))
    ss.set_walk_kernel(2)
    ss.set_mask_lanes(lpc)
    try:
        ha = _hm(ss, a.alleles, a.pos_bp, a.gpos_cm)
        hb = _hm(ss, b.alleles, a.pos_bp, a.gpos_cm)
        got = _np(ss.xpehh(ha, hb, steps=True))
    finally:
        ss.set_mask_lanes(0)
        ss.set_walk_kernel(0)
    ref = oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm)
    check_xpehh(got, ref, "xpehh lpc=%d" % lpc)


def _many_classes(seed, n1=340, n_same=200):
    """A core whose walk holds more than 64 multi-member classes at once while
    its EHH is still high: n_same identical carriers plus (n1 - n_same) / 2
    distinct identical pairs (70 by default), told apart by a 7-marker code
    right after the core."""
    rng = np.random.default_rng(seed)
    n0, M, core = 24, 160, 60
    n = n1 + n0
    npairs = (n1 - n_same) // 2
    H = (rng.random((M, n)) < 0.5).astype(np.uint8)
    H[core, :n1] = 1
    H[core, n1:] = 0
    group = np.zeros(n1, dtype=np.int64)
    group[n_same:] = 1 + (np.arange(n1 - n_same) // 2)    # the pairs, codes 1..npairs
    for direction in (+1, -1):
        for b in range(7):
            H[core + direction * (b + 1), :n1] = (group >> b) & 1
        for t in range(8, 30):                            # identical within groups for a while
            col = rng.integers(0, 2, size=npairs + 1)
            H[core + direction * t, :n1] = col[group]
    pos = (np.arange(M, dtype=np.int64) + 1) * 1000
    return H, pos, pos * 1e-6, core


@pytest.mark.parametrize("n1,n_same", [(340, 200), (230, 98), (700, 560)])
def test_ihs_more_classes_than_a_wave_row(ss, walk, n1, n_same):
    # 364 haplotypes: 8-word masks, 71 classes; 254: 4-word masks, 67 classes;
    # 724: 16-word masks two lanes a class (32 a row), 71 classes
    H, pos, gpos, core = _many_classes(3, n1, n_same)
    say("ss_ihs many classes n1=%d walk=%s" % (n1, walk))
    h = _hm(ss, H, pos, gpos)
    params = oracle.Params(maf_cutoff=0.0)
    got = _np(ss.ihs(h, ss.Params(**vars(params)), steps=True))
    ref = oracle.ihs(H, pos, gpos, params)
    check_ihs(got, ref, "many classes")
    assert ref["status"][core] in (0, 5)
    assert ref["steps"][core, 0, 1] > 8


@pytest.mark.parametrize("n1,n_same", [(340, 200), (700, 560)])
def test_xpehh_more_classes_than_a_wave_row(ss, walk, n1, n_same):
    # the two halves of the many-classes sample as populations A and B: the
    # pooled walk holds more than 64 classes at once (8-word masks at 182 +
    # 182 haplotypes, 16-word masks at 362 + 362)
    H, pos, gpos, core = _many_classes(4, n1, n_same)
    A = np.ascontiguousarray(H[:, 0::2])
    B = np.ascontiguousarray(H[:, 1::2])
    say("ss_xpehh many classes walk=%s" % walk)
    ha = _hm(ss, A, pos, gpos)
    hb = _hm(ss, B, pos, gpos)
    got = _np(ss.xpehh(ha, hb, steps=True))
    ref = oracle.xpehh(A, B, pos, gpos)
    check_xpehh(got, ref, "many classes")
    assert ref["steps"][core].max() > 8


def test_ihs_is_deterministic(ss, walk):
    d = hapgen.config_input(1)
    say("ss_ihs twice")
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    a = _np(ss.ihs(h, steps=True))
    b = _np(ss.ihs(h, steps=True))
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_ihs_large_haplotype_count(ss, walk):
    # 5000 haplotypes: 79 words per site, several waves per walk
    d = hapgen.random_haplotypes(5000, 300, 21, n_founders=100, switch_p=0.002)
    say("ss_ihs 5000 x 300")
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    got = _np(ss.ihs(h, steps=True))
    ref = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm)
    check_ihs(got, ref, "n5000")


# ---------------------------------------------------------------------------
# ss_xpehh
# ---------------------------------------------------------------------------
def test_xpehh_chr22_shaped_config(ss, walk):
    a, b = hapgen.config_input(2)
    say("ss_xpehh 204+210 x 22147 walk=%s" % walk)
    ha = _hm(ss, a.alleles, a.pos_bp, a.gpos_cm)
    hb = _hm(ss, b.alleles, b.pos_bp, b.gpos_cm)
    got = _np(ss.xpehh(ha, hb, steps=True))
    ref = oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm)
    check_xpehh(got, ref, "chr22 xpehh")


@pytest.mark.parametrize("na,nb", [(2, 2), (3, 64), (64, 65), (100, 7), (400, 300), (512, 512), (500, 524),
                                   (2500, 2500)])
def test_xpehh_ragged_populations(ss, walk, na, nb):
    M = 600 if na + nb < 2000 else 200
    a = hapgen.random_haplotypes(na, M, na, n_founders=max(2, na // 20), switch_p=0.01)
    b = hapgen.random_haplotypes(nb, M, 1000 + nb, n_founders=max(2, nb // 20), switch_p=0.02)
    say("ss_xpehh %d+%d x %d walk=%s" % (na, nb, M, walk))
    ha = _hm(ss, a.alleles, a.pos_bp, a.gpos_cm)
    hb = _hm(ss, b.alleles, a.pos_bp, a.gpos_cm)
    got = _np(ss.xpehh(ha, hb, steps=True))
    ref = oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm)
    check_xpehh(got, ref, "xpehh %d+%d" % (na, nb))


def test_xpehh_self_is_zero(ss, walk):
    a, _ = hapgen.config_input(2)
    say("ss_xpehh A vs A")
    ha = _hm(ss, a.alleles, a.pos_bp, a.gpos_cm)
    got = _np(ss.xpehh(ha, ha))
    m = np.isin(got["status"], (0, 5))
    assert m.sum() > 10000
    assert np.all(got["unstd"][m] == 0.0)
    np.testing.assert_array_equal(got["ihhA"][m], got["ihhB"][m])


@pytest.mark.parametrize("n,m", [(1, 3), (63, 17), (64, 9), (65, 130), (204, 1001), (1000, 77)])
def test_pack_matches_numpy(n, m):
    """ss_pack against its definition: bit l of word w of site s is set when
    haplotype 64 w + l carries the derived allele (any nonzero byte)."""
    import torch
    import paper_1403_6854_amd as ss
    rng = np.random.default_rng(n * 1000 + m)
    a = rng.integers(0, 2, size=(m, n), dtype=np.uint8) * rng.integers(1, 4, size=(m, n), dtype=np.uint8)
    got = ss.pack(torch.from_numpy(a).cuda()).cpu().numpy().view(np.uint64)
    W = (n + 63) // 64
    want = np.zeros((m, W), dtype=np.uint64)
    for h in range(n):
        want[:, h // 64] |= (a[:, h] != 0).astype(np.uint64) << np.uint64(h % 64)
    np.testing.assert_array_equal(got, want)


# Frequency-bin standardization takes one of several launch forms by region
# size and bin count: one workgroup per bin with the sites held in registers
# (1 to 4 rounds of 8,192) or re-read per step (up to 65,536 sites, 8 or more
# bins), or tiled partial sums (fewer bins, e.g. XPEHH's single bin, or larger
# regions); every form must agree with the oracle.
@pytest.mark.parametrize("m", [900, 12_000, 22_147, 30_000, 40_000, 70_000])
def test_standardization_forms(ss, m):
    say("ss_ihs / ss_xpehh 64 (+60) x %d standardization" % m)
    d = hapgen.copying_model(64, m, 80 * m, n_founders=12, switch_p=0.01, seed=m)
    h = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    got = _np(ss.ihs(h, steps=True))
    ref = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm)
    check_ihs(got, ref, "ihs M=%d" % m)
    assert (ref["status"] == 0).sum() > m // 4
    wide = oracle.Params(bin_width=0.25)    # 4 bins: the tiled form
    got = _np(ss.ihs(h, ss.Params(**vars(wide)), steps=True))
    ref = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, wide)
    check_ihs(got, ref, "ihs 4 bins M=%d" % m)
    e = hapgen.copying_model(60, m, 80 * m, n_founders=12, switch_p=0.01, seed=m + 1,
                             positions=(d.pos_bp, d.gpos_cm))
    hb = _hm(ss, e.alleles, d.pos_bp, d.gpos_cm)
    got = _np(ss.xpehh(h, hb, steps=True))
    ref = oracle.xpehh(d.alleles, e.alleles, d.pos_bp, d.gpos_cm)
    check_xpehh(got, ref, "xpehh M=%d" % m)


# ---------------------------------------------------------------------------
# The oracle's pinned constructions: which abort a locus reports when its two
# directions abort differently, and the pooled stop at an exact tie
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gap_side", [+1, -1])
def test_status_when_directions_abort_differently(ss, walk, gap_side):
    from tests.test_oracle_pins import _gap_one_side_edge_other
    H, pos, gpos, core = _gap_one_side_edge_other(gap_side)
    say("abort precedence, gap side %+d walk=%s" % (gap_side, walk))
    params = oracle.Params(maf_cutoff=0.0)
    got = _np(ss.ihs(_hm(ss, H, pos, gpos), ss.Params(**vars(params)), steps=True))
    ref = oracle.ihs(H, pos, gpos, params)
    check_ihs(got, ref, "ihs precedence")
    assert got["status"][core] == (3 if gap_side > 0 else 2)
    A, B = H[:, :4].copy(), H[:, 2:].copy()
    got = _np(ss.xpehh(_hm(ss, A, pos, gpos), _hm(ss, B, pos, gpos), steps=True))
    ref = oracle.xpehh(A, B, pos, gpos)
    check_xpehh(got, ref, "xpehh precedence")
    assert got["status"][core] == (3 if gap_side > 0 else 2)


def test_pooled_cutoff_tie(ss, walk):
    from tests.test_oracle_pins import _pooled_peel
    A, B, pos, gpos, core, _ = _pooled_peel(13, 12)
    say("pooled cutoff tie walk=%s" % walk)
    got = _np(ss.xpehh(_hm(ss, A, pos, gpos), _hm(ss, B, pos, gpos), steps=True))
    ref = oracle.xpehh(A, B, pos, gpos)
    check_xpehh(got, ref, "pooled tie")
    assert got["steps"][core].tolist() == [20, 20]


# ---------------------------------------------------------------------------
# Pooled XPEHH regions of 9,000 haplotypes (the served stream draws up to
# 5,000 per population): wide workgroups, thousands of classes
# ---------------------------------------------------------------------------
def pooled_pair(kind, na=5000, nb=4000, m=300):
    """(A alleles, B alleles, pos, gpos, params): a copying-model pair whose B
    shares A's founders with probability 0.8 (the served stream's regions), or
    i.i.d. alleles with a low cutoff, whose pooled walks hold thousands of
    classes before they stop."""
    if kind == "copying":
        a = hapgen.copying_model(na, m, 1580 * m, 40, 0.003, 51)
        rng = np.random.default_rng(52)
        fb = hapgen.derive_founders(rng, a.founders, 0.8)
        return a.alleles, hapgen.copy_haplotypes(rng, fb, nb, 0.003, 0.001), a.pos_bp, a.gpos_cm, oracle.Params()
    A = hapgen.random_haplotypes(na, m, 61, p=0.5)
    B = hapgen.random_haplotypes(nb, m, 62, p=0.5)
    return A.alleles, B.alleles, A.pos_bp, A.gpos_cm, oracle.Params(ehh_cutoff=2e-4)


@pytest.mark.parametrize("kind", ["copying", "iid"])
def test_xpehh_pooled_9000_haplotypes(ss, walk, kind):
    A, B, pos, gpos, params = pooled_pair(kind)
    say("ss_xpehh 5000+4000 x 300 %s walk=%s" % (kind, walk))
    got = _np(ss.xpehh(_hm(ss, A, pos, gpos), _hm(ss, B, pos, gpos), ss.Params(**vars(params)),
                       steps=True))
    ref = oracle.xpehh(A, B, pos, gpos, params)
    check_xpehh(got, ref, "xpehh 9000 %s" % kind)
    assert (ref["status"] == 0).sum() > 200


# ---------------------------------------------------------------------------
# Physical-map option: EHH integrated over base pairs, gap rules unchanged
# ---------------------------------------------------------------------------
def _gappy(n, m, seed):
    d = hapgen.random_haplotypes(n, m, seed, n_founders=max(2, n // 12), switch_p=0.01)
    rng = np.random.default_rng(seed)
    steps = rng.integers(300, 9_000, size=m)
    steps[rng.choice(m, m // 50, replace=False)] = rng.integers(20_001, 120_000, m // 50)
    steps[rng.choice(m, 4, replace=False)] = 250_000
    pos = np.cumsum(steps).astype(np.int64)
    return d, pos, pos * 1e-6


@pytest.mark.parametrize("kind", ["ihs", "xpehh"])
def test_physical_map(ss, walk, kind):
    params = oracle.Params(physical_map=1)
    if kind == "ihs":
        d = hapgen.config_input(1)
        say("ss_ihs physical map 204 x 22147 walk=%s" % walk)
        got = _np(ss.ihs(_hm(ss, d.alleles, d.pos_bp, d.gpos_cm), ss.Params(**vars(params)), steps=True))
        check_ihs(got, oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, params), "ihs physical")
        d, pos, gpos = _gappy(300, 2000, 9)
        got = _np(ss.ihs(_hm(ss, d.alleles, pos, gpos), ss.Params(**vars(params)), steps=True))
        check_ihs(got, oracle.ihs(d.alleles, pos, gpos, params), "ihs physical gaps")
    else:
        a, b = hapgen.config_input(2)
        say("ss_xpehh physical map 204+210 x 22147 walk=%s" % walk)
        got = _np(ss.xpehh(_hm(ss, a.alleles, a.pos_bp, a.gpos_cm), _hm(ss, b.alleles, a.pos_bp, a.gpos_cm),
                           ss.Params(**vars(params)), steps=True))
        check_xpehh(got, oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm, params), "xpehh physical")
        d, pos, gpos = _gappy(260, 1500, 10)
        e = hapgen.random_haplotypes(700, 1500, 11, n_founders=50, switch_p=0.01)
        got = _np(ss.xpehh(_hm(ss, d.alleles, pos, gpos), _hm(ss, e.alleles, pos, gpos),
                           ss.Params(**vars(params)), steps=True))
        check_xpehh(got, oracle.xpehh(d.alleles, e.alleles, pos, gpos, params), "xpehh physical gaps")


def test_ehh_physical_map(ss):
    d, pos, gpos = _gappy(200, 800, 12)
    dd = hapgen.HapData(d.alleles, pos, gpos)
    for core in (5, 400, 790):
        _ehh_case(ss, dd, core, oracle.Params(physical_map=1), cap=1024)


@pytest.mark.parametrize("lpc", [1, 4])
def test_mask_skip_changes_no_result(ss, lpc):
    """Batches of the bitmask walk that refine only the markers cutting a
    class give the same results as refining every marker (iHS with the
    chromosome-22 sweep, a 400-haplotype scan, and XPEHH)."""
    d = hapgen.config_input(1)
    e = hapgen.random_haplotypes(400, 2500, 77, n_founders=30, switch_p=0.004)
    a, b = hapgen.config_input(2)
    say("mask skip on/off, lanes %d" % lpc)
    hd, he = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm), _hm(ss, e.alleles, e.pos_bp, e.gpos_cm)
    hb = _hm(ss, b.alleles, a.pos_bp, a.gpos_cm)
    ss.set_walk_kernel(2)
    ss.set_mask_lanes(lpc)
    got = {}
    try:
        for skip in (0, 8, 32, 64):
            ss.set_mask_skip(skip)
            got[skip] = [_np(ss.ihs(hd, steps=True)), _np(ss.ihs(he, steps=True)),
                         _np(ss.xpehh(hd, hb, steps=True))]
    finally:
        ss.set_mask_skip(32)
        ss.set_mask_lanes(0)
        ss.set_walk_kernel(0)
    for skip in (8, 32, 64):
        for x, y in zip(got[skip], got[0]):
            for k in y:
                np.testing.assert_array_equal(x[k], y[k], err_msg="skip %d %s" % (skip, k))
    check_ihs(got[32][0], oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm), "skip chr22")
    check_xpehh(got[32][2], oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm), "skip xpehh")
