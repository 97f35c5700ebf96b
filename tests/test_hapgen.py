"""The seeded generator: shapes, determinism and the planted structure."""
import numpy as np

import hapgen


def test_config0_shape_and_determinism():
    a = hapgen.config_input(0)
    b = hapgen.config_input(0)
    assert a.alleles.shape == (2000, 200) and a.alleles.dtype == np.uint8
    np.testing.assert_array_equal(a.alleles, b.alleles)
    assert np.all(np.diff(a.pos_bp) > 0) and a.pos_bp[0] >= 1 and a.pos_bp[-1] <= 2_000_000
    np.testing.assert_array_equal(a.gpos_cm, a.pos_bp * 1e-6)
    assert set(np.unique(a.alleles)) <= {0, 1}


def test_config1_sweep_is_planted():
    d = hapgen.config_input(1)
    assert d.alleles.shape == (22147, 204)
    j = d.sweep_sites[0]
    assert abs(int(d.pos_bp[j]) - 17_500_000) < 20_000
    carriers = np.nonzero(d.alleles[j])[0]
    assert len(carriers) == round(0.7 * 204)
    lo = np.searchsorted(d.pos_bp, d.pos_bp[j] - 200_000)
    hi = np.searchsorted(d.pos_bp, d.pos_bp[j] + 200_000, side="right")
    block = d.alleles[lo:hi][:, carriers].copy()
    block[j - lo] = 1
    assert np.all(block == block[:, :1])


def test_config2_shares_sites():
    a, b = hapgen.config_input(2)
    assert a.alleles.shape == (22147, 204) and b.alleles.shape == (22147, 210)
    np.testing.assert_array_equal(a.pos_bp, b.pos_bp)
    share = (a.founders == b.founders).mean()
    assert 0.85 < share < 0.95     # 0.8 kept + 0.2 * P(redraw agrees)


def test_random_haplotypes():
    d = hapgen.random_haplotypes(10, 50, 3)
    assert d.alleles.shape == (50, 10)
    np.testing.assert_array_equal(d.pos_bp, np.arange(1, 51) * 1000)
