"""Batched scans through ss_scan_batch: the persistent walk over many regions
against the CPU oracle and against single-region calls, for every launch
configuration, under graph replay, after autotuning, and on the full
5,000 x 10^6 workload (sampled loci)."""
import sys

import numpy as np
import pytest

import hapgen
import oracle
from tests.conftest import gpu_available
from tests.test_gpu_parity import check_ihs, check_xpehh, assert_log, assert_rel

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ss():
    import paper_1403_6854_amd as ss
    ss.lib()
    yield ss
    ss.set_batch_config(ss.BatchConfig())
    ss.set_walk_kernel(0)


def _hm(ss, alleles, pos, gpos):
    import torch
    return ss.hapmat(torch.from_numpy(np.ascontiguousarray(alleles)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(pos, dtype=np.int64)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(gpos, dtype=np.float64)).cuda())


def _np(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


# (kind, n_a, n_b, n_sites, seed): iHS regions below and above 512 haplotypes,
# XPEHH regions pooled below and above 512
REGIONS = [("ihs", 120, 0, 900, 1), ("ihs", 700, 0, 1200, 2), ("xpehh", 200, 180, 800, 3),
           ("ihs", 1500, 0, 600, 4), ("xpehh", 800, 600, 700, 5), ("ihs", 333, 0, 1000, 6)]


def _data(kind, na, nb, m, seed):
    a = hapgen.random_haplotypes(na, m, seed, n_founders=max(2, na // 25), switch_p=0.004)
    if kind == "ihs":
        return a, None
    b = hapgen.random_haplotypes(nb, m, seed + 500, n_founders=max(2, nb // 25), switch_p=0.006)
    return a, b


@pytest.fixture(scope="module")
def regions(ss):
    out = []
    for kind, na, nb, m, seed in REGIONS:
        a, b = _data(kind, na, nb, m, seed)
        ha = _hm(ss, a.alleles, a.pos_bp, a.gpos_cm)
        hb = _hm(ss, b.alleles, a.pos_bp, a.gpos_cm) if b is not None else None
        if b is None:
            ref = oracle.ihs(a.alleles, a.pos_bp, a.gpos_cm)
        else:
            ref = oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm)
        out.append((kind, ha, hb, ref))
    return out


def _run_batch(ss, regions, stream=None):
    reqs = []
    for kind, ha, hb, _ in regions:
        r = ss.ScanRequest(ha, hb)
        ss.alloc_outputs(r, steps=True)
        reqs.append(r)
    ss.scan_batch(reqs, stream=stream)
    return reqs, [_np(r.out) for r in reqs]


def _check_all(got, regions, what):
    for (kind, _, _, ref), g in zip(regions, got):
        if kind == "ihs":
            check_ihs(g, ref, what)
        else:
            check_xpehh(g, ref, what)


@pytest.mark.parametrize("small_kernel", [1, 0])
def test_batch_matches_oracle_and_single_calls(ss, regions, small_kernel):
    say("ss_scan_batch %d regions small_kernel=%d" % (len(regions), small_kernel))
    ss.set_batch_config(ss.BatchConfig(small_kernel=small_kernel))
    try:
        _, got = _run_batch(ss, regions)
    finally:
        ss.set_batch_config(ss.BatchConfig())
    _check_all(got, regions, "batch")
    # bit-identical to the single-region entry points
    for (kind, ha, hb, _), g in zip(regions, got):
        one = _np(ss.ihs(ha, steps=True) if kind == "ihs" else ss.xpehh(ha, hb, steps=True))
        for k in one:
            np.testing.assert_array_equal(g[k], one[k], err_msg=kind + " " + k)


CONFIGS = [dict(threads=64), dict(threads=256), dict(threads=1024), dict(pair_cap=0), dict(pair_cap=1024),
           dict(pair_cap=8192), dict(pair_cap=16384), dict(chunk=7), dict(order=1),
           dict(blocks_per_cu=1), dict(threads=1024, pair_cap=4096, chunk=3, order=1),
           dict(small_pair_cap=1024), dict(threads=128, small_pair_cap=4096, pair_cap=0),
           dict(slots=4), dict(slots=8, chunk=4), dict(slots=4, threads=320, pair_cap=4096),
           dict(class_cap=64), dict(class_cap=0), dict(class_cap=64, pair_cap=0, slots=8),
           dict(counter_copies=1), dict(counter_copies=8), dict(counter_copies=8, class_cap=64),
           dict(kernel=1, threads=128), dict(kernel=1, threads=256), dict(kernel=1, threads=512),
           dict(kernel=1, threads=256, pair_cap=0), dict(kernel=1, threads=128, pair_cap=8192,
                                                            chunk=3, order=1)]


@pytest.mark.parametrize("cfg", CONFIGS, ids=[",".join("%s=%s" % kv for kv in c.items()) for c in CONFIGS])
def test_launch_configurations_give_identical_results(ss, regions, cfg):
    say("ss_scan_batch config %s" % cfg)
    ss.set_batch_config(ss.BatchConfig(small_kernel=0))
    try:
        _, base = _run_batch(ss, regions)
        ss.set_batch_config(ss.BatchConfig(small_kernel=0, **cfg))
        _, got = _run_batch(ss, regions)
    finally:
        ss.set_batch_config(ss.BatchConfig())
    for b, g in zip(base, got):
        for k in b:
            np.testing.assert_array_equal(g[k], b[k], err_msg=k)


def test_graph_replays_match_eager(ss, regions):
    import torch
    say("ss_scan_batch graph replay")
    reqs, eager = _run_batch(ss, regions)
    stream = torch.cuda.Stream()
    ss.set_graph(True)
    try:
        for rep in range(4):
            for r in reqs:            # eager work between replays
                for v in r.out.values():
                    v.fill_(-1 if v.dtype != torch.float64 else float("nan"))
            torch.cuda.synchronize()
            ss.scan_batch(reqs, stream=stream)
            stream.synchronize()
            got = [_np(r.out) for r in reqs]
            for e, g in zip(eager, got):
                for k in e:
                    np.testing.assert_array_equal(g[k], e[k], err_msg="replay %d %s" % (rep, k))
    finally:
        ss.set_graph(False)
        ss.graph_clear()


def test_autotune_then_parity(ss, regions):
    say("ss_autotune_batch")
    reqs = []
    for kind, ha, hb, _ in regions:
        r = ss.ScanRequest(ha, hb)
        ss.alloc_outputs(r, steps=True)
        reqs.append(r)
    ss.set_batch_config(ss.BatchConfig(small_kernel=0))
    try:
        cfg, ms, ws = ss.autotune_batch(reqs, sample_items=0)
        assert ms > 0.0
        assert cfg.kernel in (0, 1) and cfg.small_kernel == 0
        assert cfg.threads in ((64, 128, 256, 512, 1024) if cfg.kernel == 0 else (128, 256, 512))
        assert ss.get_batch_config() == cfg
        tuned = ss.group_tuning()
        say("group tuning %s" % tuned)
        for t in tuned:
            assert t["threads"] % 64 == 0 and 64 <= t["threads"] <= 1024 and t["pairs"] in (0, 1)
            assert t["counter_copies"] in (0, 1, 8) and t["chunk"] >= 1
            assert t["class_cap"] in (0, 256, 512, 1024, 2048) and 0 <= t["blocks_per_cu"] <= 4
            assert t["plain"] in (0, 1)
        ss.scan_batch(reqs, ws=ws)
        got = [_np(r.out) for r in reqs]
        # single scans by the persistent walk take the groups' settings too
        one = [_np(ss.ihs(ha, steps=True) if kind == "ihs" else ss.xpehh(ha, hb, steps=True))
               for kind, ha, hb, _ in regions]
    finally:
        ss.set_batch_config(ss.BatchConfig())
    assert ss.group_tuning() == []
    _check_all(got, regions, "tuned")
    for g, o in zip(got, one):
        for k in o:
            np.testing.assert_array_equal(g[k], o[k], err_msg=k)


def test_large_batch_full_size_sampled_parity(ss):
    """5,000 haplotypes x 10^6 sites in one persistent launch.  The oracle
    walks every 50th scored site, every 5th scored site within 200 kb of each
    sweep and the sweep sites themselves; the oracle's standardization of the
    device's scores over all 10^6 sites is compared with the device's."""
    import torch
    say("large batch: generating 5000 x 1e6 on the device")
    alleles, pos, gpos, sweeps = hapgen.large_batch_input(None, device="cuda")
    h = ss.hapmat(alleles, torch.from_numpy(pos).cuda(), torch.from_numpy(gpos).cuda())
    req = ss.ScanRequest(h)
    ss.alloc_outputs(req, steps=True)
    say("large batch: scanning")
    ss.scan_batch([req])
    got = _np(req.out)
    host = alleles.cpu().numpy()
    del alleles, h, req
    scored = np.flatnonzero(got["status"] != 1)
    near = [np.arange(*np.searchsorted(pos, [pos[s] - 200_000, pos[s] + 200_001])) for s in sweeps]
    near = np.intersect1d(np.concatenate(near), scored)[::5]
    sample = np.unique(np.concatenate([scored[::50], near, np.asarray(sweeps)]))
    say("large batch: oracle on %d sampled loci (%d near sweeps)" % (len(sample), len(near)))
    ref = oracle.ihs(host, pos, gpos, loci=sample)
    g = {k: v[sample] for k, v in got.items()}
    r = {k: v[sample] for k, v in ref.items()}
    ok_g = np.isin(g["status"], (0, 5))
    ok_r = np.isin(r["status"], (0, 5))
    np.testing.assert_array_equal(ok_g, ok_r)
    np.testing.assert_array_equal(g["status"][~ok_g], r["status"][~ok_r])
    np.testing.assert_array_equal(g["steps"], r["steps"].astype(np.int32))
    np.testing.assert_array_equal(g["freq"], r["freq"])
    every = np.ones(len(sample), dtype=bool)
    assert_rel(g["ihh1"], r["ihh1"], every, "ihh1")
    assert_rel(g["ihh0"], r["ihh0"], every, "ihh0")
    assert_log(g["unstd"], r["unstd"], every, "unstd")
    assert r["steps"].max() > 1000          # the sweeps' long walks are in the sample
    # standardization over all 10^6 sites: the oracle's routine on the
    # device's scores, bins from the derived-allele counts of the matrix
    say("large batch: oracle standardization of all sites")
    n1 = host.sum(axis=1, dtype=np.int64)
    del host
    bins = np.minimum((40 * n1) // 5000, 39).astype(np.int32)
    np.testing.assert_array_equal(bins[sample], r["bin"])
    pre = np.where(got["status"] == 5, 0, got["status"]).astype(np.int8)
    z = oracle.standardize(got["unstd"], pre, bins, 40)
    np.testing.assert_array_equal(z["status"], got["status"])
    assert_log(got["std"], z["std"], np.ones(len(pos), dtype=bool), "std")
    assert (got["status"] == 0).sum() > 100000


@pytest.mark.parametrize("cap", [64, 128])
def test_walks_that_outgrow_a_capped_class_table_are_redone(ss, cap):
    # i.i.d. alleles: the classes multiply at every marker, so most walks
    # outgrow a small table and finish in the full-table launch
    d = hapgen.random_haplotypes(900, 400, 77, p=0.5)
    e = hapgen.random_haplotypes(700, 400, 78, n_founders=40, switch_p=0.01)
    say("capped class table %d" % cap)
    ha = _hm(ss, d.alleles, d.pos_bp, d.gpos_cm)
    he = _hm(ss, e.alleles, e.pos_bp, e.gpos_cm)
    # a low cutoff keeps the i.i.d. walks going for 7+ markers (hundreds of classes)
    ref_d = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm, oracle.Params(maf_cutoff=0.0, ehh_cutoff=0.001))
    ref_e = oracle.ihs(e.alleles, e.pos_bp, e.gpos_cm)
    params = ss.Params(maf_cutoff=0.0, ehh_cutoff=0.001)
    reqs = [ss.ScanRequest(ha), ss.ScanRequest(he)]
    for r in reqs:
        ss.alloc_outputs(r, steps=True)
    try:
        ss.set_batch_config(ss.BatchConfig(small_kernel=0, class_cap=cap))
        ss.scan_batch(reqs[:1], params)
        ss.scan_batch(reqs[1:])
        got = [_np(r.out) for r in reqs]
        ss.set_batch_config(ss.BatchConfig(small_kernel=0, class_cap=0))
        ss.scan_batch(reqs[:1], params)
        full = _np(reqs[0].out)
    finally:
        ss.set_batch_config(ss.BatchConfig())
    check_ihs(got[0], ref_d, "capped iid")
    check_ihs(got[1], ref_e, "capped copying")
    for k in full:
        np.testing.assert_array_equal(got[0][k], full[k], err_msg=k)
    # the i.i.d. walks really do pass 64 classes
    assert ref_d["steps"].max() >= 7


@pytest.mark.parametrize("chunk", [1, 3])
def test_tiny_regions_leave_work_queue_parts_empty(ss, chunk):
    """Regions of 1 to 5 sites give launch groups of fewer items than the work
    queue has parts (some parts are empty from the start); every walk still
    runs once: results equal the oracle's and the single calls'."""
    specs = [("ihs", 600, 0, 1, 11), ("ihs", 700, 0, 2, 12), ("xpehh", 300, 400, 3, 13),
             ("ihs", 900, 0, 5, 14), ("xpehh", 520, 30, 4, 15)]
    regs = []
    for kind, na, nb, m, seed in specs:
        a, b = _data(kind, na, nb, m, seed)
        ha = _hm(ss, a.alleles, a.pos_bp, a.gpos_cm)
        hb = _hm(ss, b.alleles, a.pos_bp, a.gpos_cm) if b is not None else None
        ref = (oracle.ihs(a.alleles, a.pos_bp, a.gpos_cm) if b is None
               else oracle.xpehh(a.alleles, b.alleles, a.pos_bp, a.gpos_cm))
        regs.append((kind, ha, hb, ref))
    say("tiny regions, chunk %d" % chunk)
    ss.set_batch_config(ss.BatchConfig(small_kernel=0, chunk=chunk))
    try:
        _, got = _run_batch(ss, regs)
        one = [_np(ss.ihs(ha, steps=True) if kind == "ihs" else ss.xpehh(ha, hb, steps=True))
               for kind, ha, hb, _ in regs]
    finally:
        ss.set_batch_config(ss.BatchConfig())
    _check_all(got, regs, "tiny")
    for g, o in zip(got, one):
        for k in o:
            np.testing.assert_array_equal(g[k], o[k], err_msg=k)


@pytest.mark.parametrize("which", ["all", "no_pairs"])
def test_groups_walked_by_the_plain_kernel(ss, regions, which):
    """Launch groups set to the plain per-locus kernel give the results of the
    persistent walk, in batches and in single scans."""
    say("plain groups: %s" % which)
    rows = [dict(threads=t, pairs=p, counter_copies=0, class_cap=1024, chunk=1, blocks_per_cu=0, plain=1)
            for t in range(64, 1025, 64) for p in (0, 1) if which == "all" or p == 0]
    ss.set_batch_config(ss.BatchConfig(small_kernel=0))
    try:
        _, base = _run_batch(ss, regions)
        ss.set_group_tuning(rows)
        _, got = _run_batch(ss, regions)
        one = [_np(ss.ihs(ha, steps=True) if kind == "ihs" else ss.xpehh(ha, hb, steps=True))
               for kind, ha, hb, _ in regions]
    finally:
        ss.set_batch_config(ss.BatchConfig())
    _check_all(got, regions, "plain groups")
    for b, g, o in zip(base, got, one):
        for k in b:
            np.testing.assert_array_equal(g[k], b[k], err_msg=k)
            np.testing.assert_array_equal(o[k], b[k], err_msg=k)


BIG_POOLED_CONFIGS = [dict(), dict(class_cap=64), dict(class_cap=64, counter_copies=8),
                      dict(counter_copies=8, pair_cap=0), dict(class_cap=512, chunk=3),
                      dict(kernel=1, threads=512)]


@pytest.mark.parametrize("cfg", BIG_POOLED_CONFIGS,
                         ids=[",".join("%s=%s" % kv for kv in c.items()) or "default"
                              for c in BIG_POOLED_CONFIGS])
def test_batch_pooled_9000_haplotypes(ss, cfg):
    """XPEHH regions of 5,000 + 4,000 haplotypes in one batch (workgroups of
    the widest rows; with a capped class table, the full-table second launch,
    whose LDS holds one counter copy) against the oracle."""
    from tests.test_gpu_parity import pooled_pair
    regs = []
    for kind in ("copying", "iid"):
        A, B, pos, gpos, params = pooled_pair(kind)
        regs.append((_hm(ss, A, pos, gpos), _hm(ss, B, pos, gpos), params,
                     oracle.xpehh(A, B, pos, gpos, params)))
    say("ss_scan_batch 5000+4000 pooled, config %s" % cfg)
    ss.set_batch_config(ss.BatchConfig(small_kernel=0, **cfg))
    try:
        got = []
        for ha, hb, params, _ in regs:
            r = ss.ScanRequest(ha, hb)
            ss.alloc_outputs(r, steps=True)
            ss.scan_batch([r], ss.Params(**vars(params)))
            got.append(_np(r.out))
    finally:
        ss.set_batch_config(ss.BatchConfig())
    for g, (_, _, _, ref) in zip(got, regs):
        check_xpehh(g, ref, "batch pooled 9000 %s" % cfg)


# Regions above 1,024 haplotypes with a planted sweep: walks from cores in the
# sweep block run for hundreds of markers with a few large classes, the case
# the 64-marker reference passes of the class-id walk take.  (n, sites, sweep
# site, phi, first site after a gap beyond max_gap or None): sweeps in the
# middle, near the data's end (walks end at the edge inside a pass) and cut
# by a gap (walks abort inside a pass).
SWEEP_REGIONS = [(1500, 1400, 700, 0.7, None), (1300, 1200, 1120, 0.8, None),
                 (1400, 1300, 600, 0.75, 680), (2100, 900, 450, 0.9, None)]
SWEEP_CONFIGS = [dict(), dict(threads=128), dict(slots=4), dict(class_cap=64),
                 dict(pair_cap=0), dict(threads=1024, counter_copies=8)]


def _sweep_region(n, m, site, phi, gap, seed):
    d = hapgen.copying_model(n, m, 1_400_000, 30, 0.003, seed, sweeps=[(site, phi)])
    pos, gpos = d.pos_bp.copy(), d.gpos_cm.copy()
    if gap is not None:
        pos[gap:] += 300_000
        gpos[gap:] += 0.3
    return d.alleles, pos, gpos


@pytest.fixture(scope="module")
def sweep_regions(ss):
    out = []
    for i, (n, m, site, phi, gap) in enumerate(SWEEP_REGIONS):
        al, pos, gpos = _sweep_region(n, m, site, phi, gap, 40 + i)
        ref = oracle.ihs(al, pos, gpos)
        assert ref["steps"].max() >= 192, "walks too short for the reference passes"
        if gap is not None:
            assert (ref["status"] == 3).any(), "no walk aborts at the gap"
        out.append(("ihs", _hm(ss, al, pos, gpos), None, ref))
    return out


@pytest.mark.parametrize("cfg", SWEEP_CONFIGS,
                         ids=[",".join("%s=%s" % kv for kv in c.items()) or "default"
                              for c in SWEEP_CONFIGS])
def test_sweep_regions_long_walks(ss, sweep_regions, cfg):
    say("ss_scan_batch sweep regions config %s" % cfg)
    ss.set_batch_config(ss.BatchConfig(small_kernel=0, **cfg))
    try:
        _, got = _run_batch(ss, sweep_regions)
    finally:
        ss.set_batch_config(ss.BatchConfig())
    _check_all(got, sweep_regions, "sweep batch %s" % cfg)
    if not cfg:
        for (kind, ha, _, _), g in zip(sweep_regions, got):
            one = _np(ss.ihs(ha, steps=True))
            for k in one:
                np.testing.assert_array_equal(g[k], one[k], err_msg="single call " + k)


def test_gaps_at_every_offset_in_two_marker_steps(ss):
    """iHS walks over more than 1,024 haplotypes refine two markers per step;
    gaps beyond max_gap after sites of both parities make walks abort on the
    first and on the second marker of a step, and near the data's ends."""
    d = hapgen.copying_model(1100, 700, 900_000, 25, 0.01, 77)
    pos, gpos = d.pos_bp.copy(), d.gpos_cm.copy()
    for at in (90, 181, 273, 366, 460, 555):
        pos[at:] += 250_000
        gpos[at:] += 0.25
    ref = oracle.ihs(d.alleles, pos, gpos)
    assert (ref["status"] == 3).sum() > 50
    regions = [("ihs", _hm(ss, d.alleles, pos, gpos), None, ref)]
    for cfg in (dict(small_kernel=0), dict(small_kernel=0, threads=128), dict(small_kernel=0, class_cap=64)):
        say("ss_scan_batch gaps config %s" % cfg)
        ss.set_batch_config(ss.BatchConfig(**cfg))
        try:
            _, got = _run_batch(ss, regions)
        finally:
            ss.set_batch_config(ss.BatchConfig())
        _check_all(got, regions, "gaps %s" % cfg)


def test_xpehh_gaps_at_every_offset_in_two_marker_steps(ss):
    """Pooled XPEHH walks over more than 1,024 haplotypes take two markers per
    step as well (population counts in two words); gaps after sites of both
    parities end walks on either marker of a step."""
    a = hapgen.copying_model(700, 600, 800_000, 25, 0.01, 78)
    rng = np.random.default_rng(79)
    b = hapgen.copy_haplotypes(rng, hapgen.derive_founders(rng, a.founders, 0.8), 600, 0.01, 0.001)
    pos, gpos = a.pos_bp.copy(), a.gpos_cm.copy()
    for at in (75, 152, 230, 309, 389, 470):
        pos[at:] += 250_000
        gpos[at:] += 0.25
    ref = oracle.xpehh(a.alleles, b, pos, gpos)
    assert (ref["status"] == 3).sum() > 50
    regions = [("xpehh", _hm(ss, a.alleles, pos, gpos), _hm(ss, b, pos, gpos), ref)]
    for cfg in (dict(small_kernel=0), dict(small_kernel=0, counter_copies=1),
                dict(small_kernel=0, counter_copies=8, class_cap=64)):
        say("ss_scan_batch xpehh gaps config %s" % cfg)
        ss.set_batch_config(ss.BatchConfig(**cfg))
        try:
            _, got = _run_batch(ss, regions)
        finally:
            ss.set_batch_config(ss.BatchConfig())
        _check_all(got, regions, "xpehh gaps %s" % cfg)
