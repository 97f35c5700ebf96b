"""The C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments before touching the device (no compute calls, so no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("selscan_hip.h", "selscan_micro.h")]


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ss_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1403_6854_amd as ss
    if not os.path.exists(ss.LIB_PATH):
        from paper_1403_6854_amd import build
        build.build()
    return ss.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for f in ("ss_pack", "ss_workspace_bytes", "ss_ehh", "ss_ihs", "ss_xpehh", "ss_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_params_and_version(lib):
    import paper_1403_6854_amd as ss
    p = ss._Params()
    lib.ss_default_params(ctypes.byref(p))
    p.physical_map = 7
    lib.ss_default_params(ctypes.byref(p))
    assert (p.ehh_cutoff, p.maf_cutoff, p.gap_scale_bp, p.max_gap_bp, p.bin_width, p.physical_map) == \
        (0.05, 0.05, 20000, 200000, 0.025, 0)
    assert "gfx950" in ss.version()


def _desc(n_haps=204, n_sites=100, wps=4, null=False):
    import paper_1403_6854_amd as ss
    fake = 0 if null else 0x1000   # never dereferenced: the calls fail their checks first
    return ss._HapMat(fake, n_haps, n_sites, wps, fake, fake)


def test_workspace_bytes_is_host_only(lib):
    import paper_1403_6854_amd as ss
    p = ss._cparams(None)
    d = _desc()
    nb = lib.ss_workspace_bytes(ss.OP_IHS, ctypes.byref(d), None, ctypes.byref(p), 0)
    assert nb >= 100 * (1 + 4 + 32 + 8 + 16)
    assert lib.ss_workspace_bytes(ss.OP_XPEHH, ctypes.byref(d), None, ctypes.byref(p), 0) == 0
    bad = ss._cparams(ss.Params(ehh_cutoff=0.0))
    assert lib.ss_workspace_bytes(ss.OP_IHS, ctypes.byref(d), None, ctypes.byref(bad), 0) == 0


@pytest.mark.parametrize("field,value", [
    ("ehh_cutoff", 0.0), ("ehh_cutoff", 1.5), ("ehh_cutoff", float("nan")),
    ("maf_cutoff", -0.1), ("maf_cutoff", 0.6), ("gap_scale_bp", 0),
    ("max_gap_bp", 100), ("bin_width", 0.0), ("bin_width", 2.0), ("physical_map", 2),
    ("physical_map", -1)])
def test_bad_parameters_are_rejected(lib, field, value):
    import paper_1403_6854_amd as ss
    kw = {field: value}
    p = ss._cparams(ss.Params(**kw))
    d = _desc()
    x = ctypes.c_void_p(0x1000)
    rc = lib.ss_ihs(ctypes.byref(d), ctypes.byref(p), x, x, x, x, x, x, None, x, 1 << 30, None)
    assert rc == ss.SS_EARG
    assert lib.ss_last_error()


@pytest.mark.parametrize("kw", [dict(n_haps=1), dict(n_haps=40000), dict(n_sites=0),
                                dict(wps=3), dict(null=True)])
def test_bad_hapmats_are_rejected(lib, kw):
    import paper_1403_6854_amd as ss
    p = ss._cparams(None)
    d = _desc(**kw)
    x = ctypes.c_void_p(0x1000)
    rc = lib.ss_ihs(ctypes.byref(d), ctypes.byref(p), x, x, x, x, x, x, None, x, 1 << 30, None)
    assert rc == ss.SS_EARG


def test_small_workspace_and_shape_mismatch(lib):
    import paper_1403_6854_amd as ss
    p = ss._cparams(None)
    a = _desc(n_sites=100)
    b = _desc(n_sites=99)
    x = ctypes.c_void_p(0x1000)
    rc = lib.ss_ihs(ctypes.byref(a), ctypes.byref(p), x, x, x, x, x, x, None, x, 16, None)
    assert rc == ss.SS_EWS
    rc = lib.ss_xpehh(ctypes.byref(a), ctypes.byref(b), ctypes.byref(p), x, x, x, x, x, None, x,
                      1 << 30, None)
    assert rc == ss.SS_ESHAPE
    big = _desc(n_haps=20000, wps=313)
    rc = lib.ss_xpehh(ctypes.byref(big), ctypes.byref(big), ctypes.byref(p), x, x, x, x, x, None,
                      x, 1 << 30, None)
    assert rc == ss.SS_EARG
    rc = lib.ss_ehh(ctypes.byref(a), 100, ctypes.byref(p), 8, x, x, x, None, x, x, x, 1 << 20, None)
    assert rc == ss.SS_EARG        # core out of range
    rc = lib.ss_pack(None, 10, 10, 1, x, None)
    assert rc == ss.SS_EARG


def test_product_does_not_reach_the_oracle():
    # the package and its sources never import or link the test oracle
    pkg = os.path.join(ROOT, "paper_1403_6854_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "selscan_oracle" not in text, f


def _request(op, na=204, nb=210, m=100, null_out=False):
    import paper_1403_6854_amd as ss
    fake = 0x1000
    out = 0 if null_out else fake
    a = _desc(na, m, (na + 63) // 64)
    b = _desc(nb, m, (nb + 63) // 64) if op == ss.OP_XPEHH else ss._HapMat(0, 0, 0, 0, 0, 0)
    return ss._Request(op, a, b, out, out, out, out, out if op == ss.OP_IHS else 0, out, 0)


def test_batch_argument_checks_are_host_only(lib):
    import paper_1403_6854_amd as ss
    p = ss._cparams(None)
    arr = (ss._Request * 3)(_request(ss.OP_IHS), _request(ss.OP_XPEHH), _request(ss.OP_IHS, na=5000))
    single = lib.ss_workspace_bytes(ss.OP_IHS, ctypes.byref(_desc()), None, ctypes.byref(p), 0)
    nb = lib.ss_batch_workspace_bytes(arr, 3, ctypes.byref(p))
    assert nb > single
    # unknown op, empty batch, null outputs, mismatched sites
    bad = (ss._Request * 1)(_request(7))
    assert lib.ss_batch_workspace_bytes(bad, 1, ctypes.byref(p)) == 0
    assert lib.ss_scan_batch(bad, 1, ctypes.byref(p), ctypes.c_void_p(0x1000), 1 << 30, None) == ss.SS_EARG
    assert b"unknown op" in lib.ss_last_error()
    assert lib.ss_scan_batch(arr, 0, ctypes.byref(p), ctypes.c_void_p(0x1000), 1 << 30, None) == ss.SS_EARG
    nul = (ss._Request * 1)(_request(ss.OP_IHS, null_out=True))
    assert lib.ss_scan_batch(nul, 1, ctypes.byref(p), ctypes.c_void_p(0x1000), 1 << 30, None) == ss.SS_EARG
    shp = _request(ss.OP_XPEHH)
    shp.b.n_sites = 99
    one = (ss._Request * 1)(shp)
    assert lib.ss_scan_batch(one, 1, ctypes.byref(p), ctypes.c_void_p(0x1000), 1 << 30, None) == ss.SS_ESHAPE
    assert b"request 0" in lib.ss_last_error()
    # workspace too small
    good = (ss._Request * 1)(_request(ss.OP_IHS))
    assert lib.ss_scan_batch(good, 1, ctypes.byref(p), ctypes.c_void_p(0x1000), 16, None) == ss.SS_EWS


def test_batch_config_round_trip_and_range_checks(lib):
    import paper_1403_6854_amd as ss
    base = ss.get_batch_config()
    try:
        for cfg in (ss.BatchConfig(threads=320), ss.BatchConfig(kernel=1, threads=128),
                    ss.BatchConfig(pair_cap=0, small_pair_cap=4096, chunk=16, order=1,
                                   blocks_per_cu=2, small_kernel=0, slots=8, class_cap=0,
                                   counter_copies=8)):
            ss.set_batch_config(cfg)
            assert ss.get_batch_config() == cfg
        for bad in (dict(threads=96), dict(threads=2048), dict(kernel=1, threads=1024),
                    dict(kernel=2), dict(pair_cap=-1), dict(pair_cap=20000), dict(chunk=0),
                    dict(order=2), dict(small_kernel=3), dict(small_pair_cap=-5),
                    dict(blocks_per_cu=-1), dict(slots=5), dict(slots=32), dict(class_cap=10),
                    dict(class_cap=20000), dict(counter_copies=4)):
            with pytest.raises(ss.SelscanError) as e:
                ss.set_batch_config(ss.BatchConfig(**bad))
            assert e.value.code == ss.SS_EARG
    finally:
        ss.set_batch_config(base)


def test_group_tuning_is_host_only_and_cleared_by_set_config(lib):
    import ctypes
    import paper_1403_6854_amd as ss
    ss.set_batch_config(ss.get_batch_config())
    assert ss.group_tuning() == []
    n = ctypes.c_int32(-1)
    assert lib.ss_get_group_tuning(None, 0, ctypes.byref(n)) == 0 and n.value == 0
    assert lib.ss_get_group_tuning(None, 0, None) == ss.SS_EARG
    assert lib.ss_get_group_tuning(None, 3, ctypes.byref(n)) == ss.SS_EARG


def test_group_tuning_round_trip_and_range_checks(lib):
    import paper_1403_6854_amd as ss
    rows = [dict(threads=64, pairs=1, counter_copies=1, class_cap=512, chunk=2, blocks_per_cu=0, plain=0),
            dict(threads=320, pairs=0, counter_copies=8, class_cap=0, chunk=1, blocks_per_cu=3, plain=1)]
    try:
        ss.set_group_tuning(rows)
        assert ss.group_tuning() == rows
        for bad in (dict(threads=96), dict(threads=2048), dict(pairs=2), dict(counter_copies=4),
                    dict(class_cap=10), dict(chunk=0), dict(blocks_per_cu=-1), dict(plain=2)):
            with pytest.raises(ss.SelscanError) as e:
                ss.set_group_tuning([dict(rows[0], **bad)])
            assert e.value.code == ss.SS_EARG
            assert ss.group_tuning() == rows          # nothing changed
        ss.set_group_tuning([])
        assert ss.group_tuning() == []
        ss.set_group_tuning(rows)
        ss.set_batch_config(ss.get_batch_config())
        assert ss.group_tuning() == []
    finally:
        ss.set_group_tuning([])


def test_walk_kernel_choices(lib):
    import paper_1403_6854_amd as ss
    for k in (0, 1, 2, 3):
        ss.set_walk_kernel(k)
    with pytest.raises(ss.SelscanError):
        ss.set_walk_kernel(4)
    ss.set_walk_kernel(0)
    ss.set_graph(True)
    ss.set_graph(False)
    ss.graph_clear()


def test_static_scratch_entry_point_checks_before_the_device(lib):
    """ss_ihs_static refuses, on the host, null outputs and scans needing more
    scratch than its static array holds (1,000 x 300,000 here)."""
    import paper_1403_6854_amd as ss
    p = ss._cparams(None)
    fake = ctypes.c_void_p(0x1000)
    cap = lib.ss_static_scratch_bytes()
    assert cap == 32 << 20
    small = _desc(n_haps=204, n_sites=100, wps=4)
    assert lib.ss_ihs_static(ctypes.byref(small), ctypes.byref(p), fake, None, fake, fake, fake,
                             fake, None, None) == ss.SS_EARG
    big = _desc(n_haps=1000, n_sites=300_000, wps=16)
    assert lib.ss_workspace_bytes(ss.OP_IHS, ctypes.byref(big), None, ctypes.byref(p), 0) > cap
    assert lib.ss_ihs_static(ctypes.byref(big), ctypes.byref(p), fake, fake, fake, fake, fake,
                             fake, None, None) == ss.SS_EWS
    assert b"static scratch" in lib.ss_last_error()


def test_genome_standardize_checks_arguments_on_the_host(lib):
    import paper_1403_6854_amd as ss
    p = ss._cparams(None)
    x = 0x1000
    good = ss._StdRegion(x, x, x, x, 1000, 204, 0)
    arr = (ss._StdRegion * 2)(good, good)
    nb = lib.ss_genome_workspace_bytes(arr, 2, ss.OP_IHS, ctypes.byref(p))
    assert nb > 0
    cases = [
        ((ss._StdRegion * 1)(ss._StdRegion(x, None, x, x, 10, 204, 0)), ss.OP_IHS),   # iHS without freq
        ((ss._StdRegion * 1)(ss._StdRegion(x, x, x, x, 10, 1, 0)), ss.OP_IHS),      # n_haps < 2
        ((ss._StdRegion * 1)(ss._StdRegion(None, x, x, x, 10, 204, 0)), ss.OP_IHS),  # null scores
        ((ss._StdRegion * 1)(ss._StdRegion(x, x, x, x, -1, 204, 0)), ss.OP_IHS),    # negative size
        ((ss._StdRegion * 1)(good), ss.OP_EHH),                                       # not a scan op
    ]
    for regs, op in cases:
        assert lib.ss_genome_workspace_bytes(regs, 1, op, ctypes.byref(p)) == 0
        assert lib.ss_genome_standardize(regs, 1, op, ctypes.byref(p), None, ctypes.c_void_p(x),
                                         1 << 30, None) == ss.SS_EARG
    # XPEHH needs no frequencies or haplotype counts
    xp = (ss._StdRegion * 1)(ss._StdRegion(x, None, x, x, 10, 0, 0))
    assert lib.ss_genome_workspace_bytes(xp, 1, ss.OP_XPEHH, ctypes.byref(p)) > 0
    assert lib.ss_genome_standardize(arr, 2, ss.OP_IHS, ctypes.byref(p), None, ctypes.c_void_p(x),
                                     nb - 1, None) == ss.SS_EWS
    assert lib.ss_genome_standardize(arr, 0, ss.OP_IHS, ctypes.byref(p), None, ctypes.c_void_p(x),
                                     nb, None) == ss.SS_EARG


def test_measurement_kernels_check_arguments_on_the_host(lib):
    import paper_1403_6854_amd as ss
    d = ctypes.c_double(0.0)
    x = ctypes.c_void_p(0x1000)
    assert lib.ss_micro_copy(None, x, 4096, 1, None, ctypes.byref(d)) == ss.SS_EARG
    assert lib.ss_micro_copy(x, x, 4097, 1, None, ctypes.byref(d)) == ss.SS_EARG      # not a multiple of 16
    assert lib.ss_micro_copy(ctypes.c_void_p(0x1008), x, 4096, 1, None, ctypes.byref(d)) == ss.SS_EARG
    assert lib.ss_micro_valu(None, 16, 1, None, ctypes.byref(d), ctypes.byref(d)) == ss.SS_EARG
    assert lib.ss_micro_valu(x, 0, 1, None, ctypes.byref(d), ctypes.byref(d)) == ss.SS_EARG
    assert lib.ss_micro_lds_atomic(x, 16, 1, None, ctypes.byref(d), None) == ss.SS_EARG
    assert lib.ss_micro_cell(x, 0, x, 16, 1, None, ctypes.byref(d), ctypes.byref(d)) == ss.SS_EARG
    assert lib.ss_micro_cell(x, 10, x, 0, 1, None, ctypes.byref(d), ctypes.byref(d)) == ss.SS_EARG
