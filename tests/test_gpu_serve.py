"""The continuous-batching server on the GPU: every request's results in the
mix equal those of the request scanned alone, and agree with the oracle."""
import sys

import numpy as np
import pytest

import hapgen
import oracle
from tests.conftest import gpu_available
from tests.test_gpu_parity import check_ihs, check_xpehh

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _specs():
    rng = np.random.default_rng(12)
    t = np.cumsum(rng.exponential(1 / 400.0, size=24))
    out = []
    for i in range(24):
        kind = "ihs" if i % 5 not in (1, 3) else "xpehh"
        na = int(rng.choice([90, 150, 300, 520, 800, 1300]))
        nb = int(rng.choice([120, 400, 700])) if kind == "xpehh" else 0
        m = int(rng.integers(1000, 6000))
        out.append(hapgen.RequestSpec(i, kind, float(t[i]), na, nb, m, 5000 + i))
    return out


def _make(ss, spec):
    def make():
        a, b, pos, gpos = hapgen.device_region(spec, "cuda")
        ha = ss.hapmat(a, pos, gpos)
        hb = ss.hapmat(b, pos, gpos) if b is not None else None
        return ha, hb
    return make


def test_results_in_the_mix_equal_results_alone():
    import torch
    import paper_1403_6854_amd as ss
    from paper_1403_6854_amd import serve
    specs = _specs()
    reqs = [serve.ServeRequest(s.rid, s.arrival_s, s.kind,
                               serve.request_bytes(s.kind, s.n_a, s.n_b, s.n_sites), _make(ss, s),
                               s.n_sites) for s in specs]
    budget = 4 * int(np.median([r.nbytes for r in reqs]))
    say("serving %d requests, budget %d bytes" % (len(reqs), budget))
    be = serve.TorchBackend(n_streams=2, keep=None, steps=True)
    srv = serve.Server(be, budget, max_batch=6)
    done = srv.run(reqs)
    torch.cuda.synchronize()
    assert sorted(c.rid for c in done) == list(range(len(specs)))
    assert srv.batches < len(specs)           # some requests shared a batch
    assert srv.peak_bytes <= budget
    by = {c.rid: c for c in done}
    for s in specs:
        say("request %d %s n=%d/%d m=%d alone" % (s.rid, s.kind, s.n_a, s.n_b, s.n_sites))
        ha, hb = _make(ss, s)()
        alone = ss.ihs(ha, steps=True) if s.kind == "ihs" else ss.xpehh(ha, hb, steps=True)
        mixed = by[s.rid].out
        for k, v in alone.items():
            assert torch.equal(mixed[k].nan_to_num(-7.0) if v.is_floating_point() else mixed[k],
                               v.nan_to_num(-7.0) if v.is_floating_point() else v), (s.rid, k)
    # and the oracle agrees on three of them
    for s in (specs[0], specs[1], specs[5]):
        a, b, pos, gpos = hapgen.device_region(s, "cuda")
        got = {k: v.cpu().numpy() for k, v in by[s.rid].out.items()}
        if s.kind == "ihs":
            check_ihs(got, oracle.ihs(a.cpu().numpy(), pos.cpu().numpy(), gpos.cpu().numpy()),
                      "served %d" % s.rid)
        else:
            check_xpehh(got, oracle.xpehh(a.cpu().numpy(), b.cpu().numpy(), pos.cpu().numpy(),
                                          gpos.cpu().numpy()), "served %d" % s.rid)
