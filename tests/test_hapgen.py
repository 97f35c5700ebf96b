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


def test_sparse_copy_events_render_like_the_model():
    # rendering the sparse draws equals copying founders segment by segment
    rng = np.random.default_rng(3)
    F, M, n = 7, 500, 40
    fo = hapgen.draw_founders(rng, F, M)
    ev = hapgen.draw_copy_events(rng, n, M, F, 0.02, 0.01)
    got = hapgen.render_alleles(fo, ev, chunk=128).numpy()
    ref = np.empty((M, n), np.uint8)
    for h in range(n):
        f = int(ev.start[h])
        sw = dict(zip(ev.sw_site[ev.sw_hap == h].tolist(), ev.sw_step[ev.sw_hap == h].tolist()))
        for s in range(M):
            if s in sw:
                f = (f + sw[s]) % F
                assert sw[s] != 0
            ref[s, h] = fo[f, s]
        for s in ev.fl_site[ev.fl_hap == h]:
            ref[s, h] ^= 1
    np.testing.assert_array_equal(got, ref)
    assert ev.sw_site.min() >= 1 and ev.sw_site.max() < M


def test_sparse_copy_event_rates():
    rng = np.random.default_rng(11)
    n, M = 400, 20000
    ev = hapgen.draw_copy_events(rng, n, M, 50, 0.003, 0.001)
    exp_sw, exp_fl = n * (M - 1) * 0.003, n * M * 0.001
    assert abs(len(ev.sw_site) - exp_sw) < 5 * np.sqrt(exp_sw)
    assert abs(len(ev.fl_site) - exp_fl) < 5 * np.sqrt(exp_fl)
    for h in (0, 17, 399):
        s = ev.sw_site[ev.sw_hap == h]
        assert np.all(np.diff(s) > 0)


def test_large_batch_input_scaled():
    a, pos, gpos, sites = hapgen.large_batch_input(10000)
    assert tuple(a.shape) == (10000, 5000)
    assert np.all(np.diff(pos) > 0) and len(sites) == 2
    for s in sites:
        assert 0.5 * 5000 - 2 <= int(a[s].sum()) <= 0.95 * 5000 + 2
    b, pos2, _, _ = hapgen.large_batch_input(10000)
    assert np.array_equal(pos, pos2) and bool((a == b).all())


def test_request_stream():
    reqs = hapgen.request_stream(64)
    assert len(reqs) == 64 and all(a.arrival_s < b.arrival_s for a, b in zip(reqs, reqs[1:]))
    assert {r.kind for r in reqs} == {"ihs", "xpehh"}
    assert all(100 <= r.n_a <= 5000 and 1000 <= r.n_sites <= 200000 for r in reqs)


def test_hash_is_splitmix64():
    # splitmix64's published output for state 0: the finalizer applied to the
    # state after one increment
    assert int(hapgen._mix64(np.array([0], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF
    assert int(hapgen._mix64(np.array([0x9E3779B97F4A7C15], dtype=np.uint64))[0]) == 0x6E789E6AA1B965F4


def test_served_region_generator_statistics():
    spec = hapgen.RequestSpec(0, "xpehh", 0.0, 300, 250, 3000, 5)
    a, b, pos, gpos = hapgen.region_numpy(spec)
    a2, b2, pos2, _ = hapgen.region_numpy(spec)
    assert a.shape == (3000, 300) and b.shape == (3000, 250) and a.dtype == np.uint8
    assert np.array_equal(a, a2) and np.array_equal(b, b2) and np.array_equal(pos, pos2)
    assert set(np.unique(a)) <= {0, 1}
    assert pos[0] == 1 and np.all(np.diff(pos) >= 1)
    np.testing.assert_array_equal(gpos, pos * 1e-6)
    # exponential spacings of mean about bp_per_site
    g = hapgen.gaps_numpy(11, 40000, 1580)[1:]
    assert abs(g.mean() - 1579.5) < 25 and abs(np.median(g) - 1580 * np.log(2)) < 40
    # site frequencies follow the arcsine law: CDF (2/pi) asin(sqrt(p))
    xx, r = hapgen.site_p_numpy(3, 0, 20000)
    p = np.sort(xx.astype(np.float64) / r)
    cdf = 2 / np.pi * np.arcsin(np.sqrt(p))
    emp = np.arange(1, p.size + 1) / p.size
    assert np.max(np.abs(cdf - emp)) < 0.015
    # founders carry the derived allele at the site frequency
    fo = hapgen.founders_numpy(3, 0, 400, 2000)
    pp = xx[:2000].astype(np.float64) / r[:2000]
    assert np.abs(fo.mean(axis=0) - pp).max() < 0.12 and abs((fo.mean(axis=0) - pp).mean()) < 0.005
    # population B keeps A's founder entries with probability share (plus chance agreement)
    fb = hapgen.founders_numpy(3, 8, 400, 2000, fo, 0.8)
    same = (fb == fo).mean()
    assert 0.8 < same < 0.8 + 0.2 * 0.75
    # switches happen at the model's rate and always move to another founder,
    # uniformly; flips at theirs
    ident = np.repeat(np.arange(40, dtype=np.uint8)[:, None], 20000, axis=1)
    out = hapgen.copy_numpy(3, 0, ident, 300, 0.003, 0.0)
    moved = out[1:] != out[:-1]
    assert abs(moved.mean() - 0.003) < 0.0004
    step = ((out[1:].astype(int) - out[:-1].astype(int)) % 40)[moved]
    assert step.min() >= 1 and np.bincount(step, minlength=40)[1:].min() > 0.5 * moved.sum() / 39
    assert np.bincount(out[0], minlength=40).min() > 0     # starting founders cover all 40
    zero = np.zeros((40, 20000), dtype=np.uint8)
    fl = hapgen.copy_numpy(3, 0, zero, 300, 0.003, 0.001)
    assert abs(fl.mean() - 0.001) < 0.0002
