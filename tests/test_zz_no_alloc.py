"""ss_ihs_static (the iHS scan with its scratch in the library's static device
array, for callers that cannot allocate) against ss_ihs with a workspace,
through the C ABI: identical results on two calls in a row, the second on a
smaller input, so that what the first call left in the shared array cannot
leak into the second; and against the oracle."""
import sys

import numpy as np
import pytest

import hapgen
import oracle
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _hm(ss, d):
    import torch
    return ss.hapmat(torch.from_numpy(np.ascontiguousarray(d.alleles)).cuda(),
                     torch.from_numpy(d.pos_bp).cuda(), torch.from_numpy(d.gpos_cm).cuda())


def _np(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("inputs", ["mask_walk", "persistent_walk"])
def test_static_scratch_equals_workspace_entry_point(inputs):
    import paper_1403_6854_amd as ss
    from tests.test_gpu_parity import check_ihs
    if inputs == "mask_walk":     # 204 x 22,147 then 150 x 1,500: the bitmask walk
        big, small = hapgen.config_input(1), hapgen.random_haplotypes(150, 1500, 3, n_founders=12,
                                                                      switch_p=0.01)
    else:                         # 700 x 1,200 then 600 x 700: the persistent walk
        big = hapgen.random_haplotypes(700, 1200, 2, n_founders=28, switch_p=0.004)
        small = hapgen.random_haplotypes(600, 700, 5, n_founders=24, switch_p=0.004)
    assert ss.workspace_bytes(ss.OP_IHS, _hm(ss, big)) <= ss.static_scratch_bytes()
    for name, d in (("first", big), ("second, smaller", small)):
        say("ss_ihs_static %s call: %d x %d" % (name, d.n_haps, d.n_sites))
        h = _hm(ss, d)
        got = _np(ss.ihs_static(h, steps=True))
        want = _np(ss.ihs(h, steps=True))
        for k in want:
            np.testing.assert_array_equal(got[k], want[k], err_msg="%s call, %s" % (name, k))
        check_ihs(got, oracle.ihs(d.alleles, d.pos_bp, d.gpos_cm), "static scratch, " + name)
