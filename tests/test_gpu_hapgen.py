"""The served requests' generator on the GPU (hapgen/gen.hip) gives the same
positions and alleles as its numpy mirror."""
import sys

import numpy as np
import pytest

import hapgen
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

SPECS = [hapgen.RequestSpec(0, "ihs", 0.0, 100, 0, 1000, 11),
         hapgen.RequestSpec(1, "xpehh", 0.0, 300, 250, 3001, 12),
         hapgen.RequestSpec(2, "xpehh", 0.0, 63, 129, 4099, 13),
         hapgen.RequestSpec(3, "ihs", 0.0, 1, 0, 65, 14)]


@pytest.mark.parametrize("spec", SPECS, ids=[str(s.rid) for s in SPECS])
def test_device_generator_matches_numpy(spec):
    import torch
    print("device_region %s" % (spec,), flush=True)
    sys.stdout.flush()
    a, b, pos, gpos = hapgen.device_region(spec, "cuda")
    torch.cuda.synchronize()
    ra, rb, rpos, rgpos = hapgen.region_numpy(spec)
    np.testing.assert_array_equal(pos.cpu().numpy(), rpos)
    np.testing.assert_array_equal(gpos.cpu().numpy(), rgpos)
    np.testing.assert_array_equal(a.cpu().numpy(), ra)
    if spec.kind == "xpehh":
        np.testing.assert_array_equal(b.cpu().numpy(), rb)
    else:
        assert b is None and rb is None
