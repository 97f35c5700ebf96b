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


def test_device_request_generator():
    import torch
    reqs = hapgen.request_stream(64)
    assert len(reqs) == 64 and all(a.arrival_s < b.arrival_s for a, b in zip(reqs, reqs[1:]))
    assert {r.kind for r in reqs} == {"ihs", "xpehh"}
    assert all(100 <= r.n_a <= 5000 and 1000 <= r.n_sites <= 200000 for r in reqs)
    spec = hapgen.RequestSpec(0, "xpehh", 0.0, 300, 250, 3000, 5)
    a, b, pos, gpos = hapgen.device_region(spec, "cpu")
    a2, b2, pos2, _ = hapgen.device_region(spec, "cpu")
    assert tuple(a.shape) == (3000, 300) and tuple(b.shape) == (3000, 250)
    assert bool((a == a2).all()) and bool((b == b2).all()) and bool((pos == pos2).all())
    assert bool((pos[1:] > pos[:-1]).all())
    # switches happen at the model's rate and always move to another founder
    gen = torch.Generator()
    gen.manual_seed(3)
    fo = torch.arange(40, dtype=torch.uint8)[:, None].expand(40, 20000).contiguous()
    out = hapgen._device_copy(gen, fo, 300, 0.003, 0.0)
    rate = (out[1:] != out[:-1]).float().mean().item()
    assert abs(rate - 0.003) < 0.0004
