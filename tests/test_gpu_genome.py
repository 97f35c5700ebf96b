"""Genome-wide standardization (Eq. 6 and Eq. 9 over the whole genome): the
scores of several scans standardized together by ss_genome_standardize,
against the oracle's standardization of the concatenated loci."""
import sys

import numpy as np
import pytest

import hapgen
import oracle
from tests.conftest import gpu_available
from tests.test_gpu_parity import assert_log, check_ihs, check_xpehh

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ss():
    import paper_1403_6854_amd as ss
    ss.lib()
    return ss


def _hm(ss, alleles, pos, gpos):
    import torch
    return ss.hapmat(torch.from_numpy(np.ascontiguousarray(alleles)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(pos, dtype=np.int64)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(gpos, dtype=np.float64)).cuda())


def _np(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check_genome(gpu_outs, ref_outs, binstat, nbins, what):
    res, stats = oracle.genome_standardize(ref_outs, nbins)
    for i, (g, r) in enumerate(zip(gpu_outs, res)):
        g = _np(g)
        np.testing.assert_array_equal(g["status"], r["status"], err_msg="%s scan %d status" % (what, i))
        assert_log(g["std"], r["std"], np.ones(len(r["std"]), dtype=bool), "%s scan %d std" % (what, i))
    bs = binstat.cpu().numpy()
    np.testing.assert_array_equal(bs[:, 0], stats["n"].astype(np.float64))
    f = stats["n"] >= 1
    assert_log(bs[f, 1], stats["mean"][f], np.ones(int(f.sum()), dtype=bool), what + " mean")
    f = stats["n"] >= 2
    assert_log(bs[f, 2], stats["sd"][f], np.ones(int(f.sum()), dtype=bool), what + " sd")
    return res


# (kind, haplotypes, sites, founders, switch rate); the tiny scan's walks are
# short and its bins hold one locus or none, so alone it has BIN statuses
IHS_SCANS = [("chr22", 204, 22147, 0, 0.0), ("copying", 150, 3000, 7, 0.008),
             ("persistent", 600, 2000, 30, 0.008), ("tiny", 50, 120, 6, 0.1)]


def _ihs_inputs():
    out = []
    for kind, n, m, nf, sw in IHS_SCANS:
        d = hapgen.config_input(1) if kind == "chr22" else hapgen.random_haplotypes(
            n, m, n + m, n_founders=nf, switch_p=sw)
        out.append(d)
    return out


def test_genome_standardization_of_ihs_scans(ss):
    ins = _ihs_inputs()
    gpu, ref = [], []
    for d in ins:
        say("ss_ihs %d x %d for the genome" % (d.n_haps, d.n_sites))
        o = ss.ihs(_hm(ss, d.alleles, d.pos_bp, d.gpos_cm), steps=True)
        r = oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm)
        check_ihs(_np(o), r, "scan alone")
        gpu.append(o)
        ref.append(r)
    assert any((r["status"] == 5).any() for r in ref)   # the tiny scan's bins are too small alone
    say("ss_genome_standardize over %d iHS scans" % len(gpu))
    bs = ss.genome_standardize(gpu, [d.n_haps for d in ins])
    res = _check_genome(gpu, ref, bs, 40, "ihs genome")
    # the genome-wide scores differ from the per-scan ones
    assert not np.array_equal(np.nan_to_num(res[1]["std"]), np.nan_to_num(ref[1]["std"]))
    # repeating the call gives the same bits
    again = [{k: v.clone() for k, v in o.items()} for o in gpu]
    ss.genome_standardize(again, [d.n_haps for d in ins])
    for a, b in zip(again, gpu):
        for k in ("std", "status"):
            np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy())


def test_genome_standardization_of_xpehh_scans(ss):
    gpu, ref = [], []
    a, b = hapgen.config_input(2)
    pairs = [(a, b)]
    for na, nb, m, seed in ((300, 250, 1500, 5), (40, 30, 200, 6)):
        x = hapgen.random_haplotypes(na, m, seed, n_founders=12, switch_p=0.01)
        y = hapgen.random_haplotypes(nb, m, seed + 50, n_founders=10, switch_p=0.01)
        pairs.append((x, y))
    for x, y in pairs:
        say("ss_xpehh %d+%d x %d for the genome" % (x.n_haps, y.n_haps, x.n_sites))
        o = ss.xpehh(_hm(ss, x.alleles, x.pos_bp, x.gpos_cm), _hm(ss, y.alleles, x.pos_bp, x.gpos_cm),
                     steps=True)
        r = oracle.xpehh(x.alleles, y.alleles, x.pos_bp, x.gpos_cm)
        check_xpehh(_np(o), r, "pair alone")
        gpu.append(o)
        ref.append(r)
    say("ss_genome_standardize over %d XPEHH scans" % len(gpu))
    bs = ss.genome_standardize(gpu, op=ss.OP_XPEHH)
    _check_genome(gpu, ref, bs, 1, "xpehh genome")


def test_genome_standardization_of_a_batch(ss):
    from tests.test_gpu_batch import REGIONS, _data
    reqs, refs, kinds, ns = [], [], [], []
    for kind, na, nb, m, seed in REGIONS:
        x, y = _data(kind, na, nb, m, seed)
        r = ss.ScanRequest(_hm(ss, x.alleles, x.pos_bp, x.gpos_cm),
                           _hm(ss, y.alleles, x.pos_bp, x.gpos_cm) if y is not None else None)
        ss.alloc_outputs(r, steps=True)
        reqs.append(r)
        refs.append(oracle.ihs(x.alleles, x.pos_bp, x.gpos_cm) if y is None
                    else oracle.xpehh(x.alleles, y.alleles, x.pos_bp, x.gpos_cm))
        kinds.append(kind)
        ns.append(na)
    say("ss_scan_batch then ss_genome_standardize")
    ss.scan_batch(reqs)
    ihs = [i for i, k in enumerate(kinds) if k == "ihs"]
    xp = [i for i, k in enumerate(kinds) if k == "xpehh"]
    bs = ss.genome_standardize([reqs[i].out for i in ihs], [ns[i] for i in ihs])
    _check_genome([reqs[i].out for i in ihs], [refs[i] for i in ihs], bs, 40, "batch ihs genome")
    bs = ss.genome_standardize([reqs[i].out for i in xp], op=ss.OP_XPEHH)
    _check_genome([reqs[i].out for i in xp], [refs[i] for i in xp], bs, 1, "batch xpehh genome")
