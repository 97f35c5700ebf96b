"""Seeded synthetic haplotype data for EHH / iHS / XPEHH scans.

This module only draws random inputs: positions, a genetic map and 0/1
haplotypes from a founder-copying model.  It holds none of the scan's
arithmetic (no class counts, no EHH, no integration, no statistics), so the
CPU oracle and the GPU path can both take their inputs from here without
sharing any of the method.

Allele encoding follows the paper's EHH section: 0 is the ancestral allele
and 1 the derived allele.  Matrices are site-major: ``alleles[site, hap]``.

Copying model (stands in for the paper's 1000 Genomes chr22 and ms data,
which are not available):
  * positions: ``n_sites`` distinct integers drawn uniformly without
    replacement from ``[1, length_bp]``, sorted; genetic map 1 cM/Mb, so
    ``gpos_cm = pos_bp * 1e-6``;
  * founders: per site an allele frequency ``p ~ Beta(0.5, 0.5)`` and
    ``n_founders`` founder alleles ``~ Bernoulli(p)``;
  * haplotypes: each starts on a uniformly chosen founder, switches to a
    uniformly chosen *other* founder with probability ``switch_p`` before each
    next site, copies that founder's allele, and finally every allele flips
    with probability ``flip_p``;
  * planted sweeps (after the flips): ``round(phi * n)`` carriers chosen
    uniformly take the first carrier's alleles at every site within
    ``block_bp/2`` of the sweep site; at the sweep site itself carriers get 1
    and everyone else 0;
  * a second population shares each (founder, site) entry with the first
    population's founders with probability ``share_p`` and otherwise redraws
    it from ``Bernoulli(p')`` with a fresh per-site ``p' ~ Beta(0.5, 0.5)``.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "HapData", "draw_positions", "draw_founders", "derive_founders",
    "copy_haplotypes", "plant_sweep", "copying_model", "config_input",
    "random_haplotypes", "CONFIGS", "CopyEvents", "draw_copy_events", "render_alleles",
    "plant_sweep_tensor", "large_batch_input", "poisson_arrivals", "log_uniform_int",
    "SERVE", "RequestSpec", "request_stream", "device_region", "region_numpy", "build_gpu",
]


@dataclasses.dataclass
class HapData:
    alleles: np.ndarray          # uint8 [n_sites, n_haps]
    pos_bp: np.ndarray           # int64 [n_sites], strictly increasing here
    gpos_cm: np.ndarray          # float64 [n_sites]
    founders: Optional[np.ndarray] = None   # uint8 [n_founders, n_sites]
    sweep_sites: tuple = ()

    @property
    def n_haps(self) -> int:
        return int(self.alleles.shape[1])

    @property
    def n_sites(self) -> int:
        return int(self.alleles.shape[0])


def draw_positions(rng: np.random.Generator, n_sites: int, length_bp: int):
    if n_sites > length_bp:
        raise ValueError("more sites than base pairs")
    pos = np.sort(rng.choice(length_bp, size=n_sites, replace=False)).astype(np.int64) + 1
    gpos = pos.astype(np.float64) * 1e-6
    return pos, gpos


def draw_founders(rng: np.random.Generator, n_founders: int, n_sites: int) -> np.ndarray:
    p = rng.beta(0.5, 0.5, size=n_sites)
    return (rng.random((n_founders, n_sites)) < p[None, :]).astype(np.uint8)


def derive_founders(rng: np.random.Generator, base: np.ndarray, share_p: float) -> np.ndarray:
    n_founders, n_sites = base.shape
    p_new = rng.beta(0.5, 0.5, size=n_sites)
    fresh = (rng.random((n_founders, n_sites)) < p_new[None, :]).astype(np.uint8)
    keep = rng.random((n_founders, n_sites)) < share_p
    return np.where(keep, base, fresh).astype(np.uint8)


def copy_haplotypes(rng: np.random.Generator, founders: np.ndarray, n_haps: int,
                    switch_p: float, flip_p: float, chunk: int = 16384) -> np.ndarray:
    """Founder-copying haplotypes, returned site-major uint8 [n_sites, n_haps].

    Sites are produced in chunks so that large configurations never hold an
    n_haps x n_sites integer path array; the copied founder is carried across
    chunk boundaries.
    """
    n_founders, n_sites = founders.shape
    out = np.empty((n_sites, n_haps), dtype=np.uint8)
    cur = rng.integers(0, n_founders, size=n_haps).astype(np.int64)
    hap_idx = np.arange(n_haps)
    for s0 in range(0, n_sites, chunk):
        s1 = min(n_sites, s0 + chunk)
        w = s1 - s0
        # switch before every site except the very first one
        sw = rng.random((w, n_haps)) < switch_p
        if s0 == 0:
            sw[0, :] = False
        step = rng.integers(1, max(2, n_founders), size=(w, n_haps)).astype(np.int64)
        if n_founders < 2:
            step[:] = 0
        step *= sw
        path = (cur[None, :] + np.cumsum(step, axis=0)) % n_founders
        cur = path[-1].copy()
        block = founders[path, (np.arange(s0, s1))[:, None]]
        flips = rng.random((w, n_haps)) < flip_p
        out[s0:s1] = block ^ flips.astype(np.uint8)
        del sw, step, path, block, flips
    del hap_idx
    return out


@dataclasses.dataclass
class CopyEvents:
    """The copying model's random draws in sparse form, for large matrices.

    The same model as :func:`copy_haplotypes` (a Bernoulli(switch_p) switch
    before every site after the first, a Bernoulli(flip_p) flip of every
    allele), drawn per haplotype as event lists instead of one uniform per
    (site, haplotype): given its count K ~ Binomial(m, p), the set of sites
    where a Bernoulli(p) process fires is a uniform K-subset.
    """
    n_haps: int
    n_sites: int
    n_founders: int
    start: np.ndarray     # int64 [n_haps] founder copied at site 0
    sw_hap: np.ndarray    # int64 [K] haplotype of each switch
    sw_site: np.ndarray   # int64 [K] site from which the new founder is copied (>= 1)
    sw_step: np.ndarray   # int64 [K] new founder = (old + step) mod n_founders, step in [1, F-1]
    fl_hap: np.ndarray    # int64 [K'] haplotype of each flipped allele
    fl_site: np.ndarray   # int64 [K'] its site


def _subsets(rng: np.random.Generator, counts: np.ndarray, m: int, offset: int) -> np.ndarray:
    parts = [np.sort(rng.choice(m, size=int(k), replace=False)) + offset if k else
             np.empty(0, dtype=np.int64) for k in counts]
    return np.concatenate(parts).astype(np.int64) if parts else np.empty(0, dtype=np.int64)


def draw_copy_events(rng: np.random.Generator, n_haps: int, n_sites: int, n_founders: int,
                     switch_p: float, flip_p: float) -> CopyEvents:
    start = rng.integers(0, n_founders, size=n_haps).astype(np.int64)
    ks = rng.binomial(max(0, n_sites - 1), switch_p, size=n_haps) if n_sites > 1 \
        else np.zeros(n_haps, dtype=np.int64)
    sw_site = _subsets(rng, ks, max(1, n_sites - 1), 1)
    sw_hap = np.repeat(np.arange(n_haps, dtype=np.int64), ks)
    if n_founders >= 2:
        sw_step = rng.integers(1, n_founders, size=len(sw_site)).astype(np.int64)
    else:
        sw_step = np.zeros(len(sw_site), dtype=np.int64)
    kf = rng.binomial(n_sites, flip_p, size=n_haps)
    fl_site = _subsets(rng, kf, n_sites, 0)
    fl_hap = np.repeat(np.arange(n_haps, dtype=np.int64), kf)
    return CopyEvents(n_haps, n_sites, n_founders, start, sw_hap, sw_site, sw_step, fl_hap, fl_site)


def render_alleles(founders: np.ndarray, ev: CopyEvents, device="cpu", chunk: int = 65536):
    """The site-major uint8 allele matrix of a CopyEvents draw, as a torch
    tensor on ``device`` (integer operations only, so every device gives the
    same matrix)."""
    import torch
    F, M = founders.shape
    n = ev.n_haps
    fd = torch.from_numpy(np.ascontiguousarray(founders)).to(device)
    out = torch.empty((M, n), dtype=torch.uint8, device=device)
    order = np.argsort(ev.sw_site, kind="stable")
    sites, haps, steps = ev.sw_site[order], ev.sw_hap[order], ev.sw_step[order]
    cur = torch.from_numpy(ev.start).to(device)
    for s0 in range(0, M, chunk):
        s1 = min(M, s0 + chunk)
        i0, i1 = np.searchsorted(sites, [s0, s1])
        delta = torch.zeros((s1 - s0, n), dtype=torch.int64, device=device)
        if i1 > i0:
            delta[torch.from_numpy(sites[i0:i1] - s0).to(device),
                  torch.from_numpy(haps[i0:i1]).to(device)] = torch.from_numpy(steps[i0:i1]).to(device)
        path = torch.remainder(cur[None, :] + torch.cumsum(delta, dim=0), F)
        cur = path[-1].clone()
        col = torch.arange(s0, s1, device=device)[:, None]
        out[s0:s1] = fd[path, col]
        del delta, path
    if len(ev.fl_site):
        fs = torch.from_numpy(ev.fl_site).to(device)
        fh = torch.from_numpy(ev.fl_hap).to(device)
        out[fs, fh] = out[fs, fh] ^ 1
    return out


def plant_sweep_tensor(rng: np.random.Generator, alleles, pos_bp: np.ndarray, site: int,
                       phi: float, block_bp: int = 400_000) -> None:
    """:func:`plant_sweep` on a torch allele matrix (same draws, same result)."""
    import torch
    n_haps = alleles.shape[1]
    k = int(round(phi * n_haps))
    carriers = rng.choice(n_haps, size=k, replace=False)
    lo = int(np.searchsorted(pos_bp, pos_bp[site] - block_bp // 2, side="left"))
    hi = int(np.searchsorted(pos_bp, pos_bp[site] + block_bp // 2, side="right"))
    ct = torch.from_numpy(carriers.astype(np.int64)).to(alleles.device)
    if k > 0:
        template = alleles[lo:hi, int(carriers[0])].clone()
        alleles[lo:hi, ct] = template[:, None].expand(hi - lo, k)
    alleles[site, :] = 0
    alleles[site, ct] = 1


def plant_sweep(rng: np.random.Generator, alleles: np.ndarray, pos_bp: np.ndarray,
                site: int, phi: float, block_bp: int = 400_000) -> None:
    n_haps = alleles.shape[1]
    k = int(round(phi * n_haps))
    carriers = rng.choice(n_haps, size=k, replace=False)
    lo = np.searchsorted(pos_bp, pos_bp[site] - block_bp // 2, side="left")
    hi = np.searchsorted(pos_bp, pos_bp[site] + block_bp // 2, side="right")
    if k > 0:
        template = alleles[lo:hi, carriers[0]].copy()
        alleles[lo:hi, carriers] = template[:, None]
    alleles[site, :] = 0
    alleles[site, carriers] = 1


def copying_model(n_haps: int, n_sites: int, length_bp: int, n_founders: int,
                  switch_p: float, seed: int, flip_p: float = 0.001,
                  sweeps: Sequence = (), founders: Optional[np.ndarray] = None,
                  positions=None) -> HapData:
    """One population from the copying model (see module docstring).

    ``sweeps`` is a sequence of ``(site_index, phi)``; ``founders`` and
    ``positions`` let a second population reuse the first one's sites.
    """
    rng = np.random.default_rng(seed)
    if positions is None:
        pos, gpos = draw_positions(rng, n_sites, length_bp)
    else:
        pos, gpos = positions
    if founders is None:
        founders = draw_founders(rng, n_founders, n_sites)
    alleles = copy_haplotypes(rng, founders, n_haps, switch_p, flip_p)
    for site, phi in sweeps:
        plant_sweep(rng, alleles, pos, int(site), float(phi))
    return HapData(alleles=alleles, pos_bp=pos, gpos_cm=gpos, founders=founders,
                   sweep_sites=tuple(int(s) for s, _ in sweeps))


# ---------------------------------------------------------------------------
# The workload shapes.  Index i uses seed 1000 + i.
# ---------------------------------------------------------------------------
CONFIGS = {
    0: dict(name="ihs_tiny_200x2000", n_haps=200, n_sites=2000, length_bp=2_000_000,
            n_founders=20, switch_p=0.01),
    1: dict(name="ihs_chr22_204x22147", n_haps=204, n_sites=22147, length_bp=35_000_000,
            n_founders=40, switch_p=0.003, sweep_phi=0.7, sweep_at_bp=17_500_000),
    2: dict(name="xpehh_chr22_204+210x22147", n_haps_b=210, share_p=0.8),
    3: dict(name="ihs_batched_5000x1e6", n_haps=5000, n_sites=1_000_000,
            length_bp=250_000_000, n_founders=200, switch_p=0.001, n_sweeps=20,
            phi_range=(0.5, 0.95)),
}


def _nearest_site(pos: np.ndarray, bp: int) -> int:
    i = int(np.searchsorted(pos, bp))
    if i >= len(pos):
        return len(pos) - 1
    if i > 0 and abs(int(pos[i - 1]) - bp) <= abs(int(pos[i]) - bp):
        return i - 1
    return i


def config_input(idx: int, scale_sites: Optional[int] = None):
    """Inputs for workload ``idx``.

    Returns a HapData for 0, 1 and 3, and a pair (A, B) for 2.
    ``scale_sites`` shrinks configuration 3 to fewer sites (same density and
    haplotype count) for tests that cannot hold the full matrix.
    """
    if idx == 0:
        c = CONFIGS[0]
        return copying_model(c["n_haps"], c["n_sites"], c["length_bp"], c["n_founders"],
                             c["switch_p"], seed=1000)
    if idx == 1:
        c = CONFIGS[1]
        rng = np.random.default_rng(1001)
        pos, gpos = draw_positions(rng, c["n_sites"], c["length_bp"])
        founders = draw_founders(rng, c["n_founders"], c["n_sites"])
        j = _nearest_site(pos, c["sweep_at_bp"])
        alleles = copy_haplotypes(rng, founders, c["n_haps"], c["switch_p"], 0.001)
        plant_sweep(rng, alleles, pos, j, c["sweep_phi"])
        return HapData(alleles, pos, gpos, founders, (j,))
    if idx == 2:
        a = config_input(1)
        c1, c2 = CONFIGS[1], CONFIGS[2]
        rng = np.random.default_rng(1002)
        fb = derive_founders(rng, a.founders, c2["share_p"])
        alleles = copy_haplotypes(rng, fb, c2["n_haps_b"], c1["switch_p"], 0.001)
        b = HapData(alleles, a.pos_bp, a.gpos_cm, fb, ())
        return a, b
    if idx == 3:
        alleles, pos, gpos, sites = large_batch_input(scale_sites, device="cpu")
        return HapData(alleles.numpy(), pos, gpos, None, sites)
    raise KeyError(idx)


def large_batch_input(scale_sites: Optional[int] = None, device="cpu"):
    """The 5,000-haplotype x 10^6-site workload (seed 1003), built with the
    sparse copying-model draws and rendered on ``device``: returns (alleles
    torch uint8 [M, n], pos_bp, gpos_cm, sweep sites).  ``scale_sites`` keeps
    the density and haplotype count on fewer sites."""
    c = CONFIGS[3]
    m = c["n_sites"] if scale_sites is None else int(scale_sites)
    length = c["length_bp"] if scale_sites is None else max(m, int(c["length_bp"] * m / c["n_sites"]))
    rng = np.random.default_rng(1003)
    pos, gpos = draw_positions(rng, m, length)
    founders = draw_founders(rng, c["n_founders"], m)
    ev = draw_copy_events(rng, c["n_haps"], m, c["n_founders"], c["switch_p"], 0.001)
    alleles = render_alleles(founders, ev, device=device)
    del founders, ev
    n_sw = c["n_sweeps"] if scale_sites is None else max(1, min(c["n_sweeps"], m // 5000))
    sites = [int((k + 0.5) * m / n_sw) for k in range(n_sw)]
    phis = rng.uniform(*c["phi_range"], size=n_sw)
    for s, phi in zip(sites, phis):
        plant_sweep_tensor(rng, alleles, pos, s, float(phi))
    return alleles, pos, gpos, tuple(sites)


def random_haplotypes(n_haps: int, n_sites: int, seed: int, p: float = 0.5,
                      spacing_bp: int = 1000, n_founders: int = 0,
                      switch_p: float = 0.05) -> HapData:
    """Small inputs for tests: i.i.d. Bernoulli(p) alleles (``n_founders == 0``)
    or a small copying model, on evenly spaced sites (``spacing_bp`` apart)."""
    rng = np.random.default_rng(seed)
    pos = (np.arange(n_sites, dtype=np.int64) + 1) * int(spacing_bp)
    gpos = pos.astype(np.float64) * 1e-6
    if n_founders <= 0:
        alleles = (rng.random((n_sites, n_haps)) < p).astype(np.uint8)
        return HapData(alleles, pos, gpos)
    founders = draw_founders(rng, n_founders, n_sites)
    alleles = copy_haplotypes(rng, founders, n_haps, switch_p, 0.001)
    return HapData(alleles, pos, gpos, founders)


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


# ---------------------------------------------------------------------------
# Served region-scan requests: many regions of random sizes, generated on the
# device from per-request seeds with counter-based hashes, so that a request
# stream of ~10^11 alleles does not wait on the host.
# ---------------------------------------------------------------------------
SERVE = dict(n_requests=4096, rate_per_s=200.0, p_ihs=0.6, n_range=(100, 5000),
             sites_range=(1000, 200_000), bp_per_site=1580, n_founders=40, switch_p=0.003,
             flip_p=0.001, share_p=0.8, arrival_seed=7, seed_base=1 << 20)


@dataclasses.dataclass
class RequestSpec:
    rid: int
    kind: str          # "ihs" or "xpehh"
    arrival_s: float
    n_a: int
    n_b: int           # 0 for iHS
    n_sites: int
    seed: int


def request_stream(n_requests: Optional[int] = None, rate_per_s: Optional[float] = None):
    """The served workload: Poisson arrivals, iHS with probability p_ihs else
    XPEHH, haplotype counts per population and site counts log-uniform."""
    c = SERVE
    n = c["n_requests"] if n_requests is None else int(n_requests)
    rate = c["rate_per_s"] if rate_per_s is None else float(rate_per_s)
    arr = poisson_arrivals(n, rate, seed=c["arrival_seed"])
    rng = np.random.default_rng(c["arrival_seed"] + 1)
    out = []
    for r in range(n):
        kind = "ihs" if rng.random() < c["p_ihs"] else "xpehh"
        na = log_uniform_int(rng, *c["n_range"])
        nb = log_uniform_int(rng, *c["n_range"]) if kind == "xpehh" else 0
        m = log_uniform_int(rng, *c["sites_range"])
        out.append(RequestSpec(r, kind, float(arr[r]), na, nb, m, c["seed_base"] + r))
    return out


# The served requests' generator: counter-based hashes (splitmix64's
# finalizer over key ^ (row << 32 | column)), evaluated by the HIP kernels in
# gen.hip on the device and by the numpy functions below on the host; both
# take the same integer and float32 steps, so they give the same arrays.
# Stream tags per population: 0 (A) or 8 (B) plus 0 site frequency, 1 founder
# alleles, 2 sharing with A, 3 switches and flips, 5 starting founder; 15 the
# site spacings.
HERE = os.path.dirname(os.path.abspath(__file__))
GEN_LIB = os.path.join(HERE, "libhapgen_gpu.so")
_U64 = np.uint64
_F32 = np.float32


def _mix64(z):
    z = np.asarray(z, dtype=_U64)
    with np.errstate(over="ignore"):
        z = z + _U64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
    return z ^ (z >> _U64(31))


def _key(seed: int, tag: int) -> int:
    return int(_mix64(np.array([(int(seed) * 16 + int(tag)) % (1 << 64)], dtype=_U64))[0])


def _draw(key: int, row, col):
    row = np.asarray(row, dtype=_U64)
    col = np.asarray(col, dtype=_U64)
    return _mix64(_U64(key) ^ ((row << _U64(32)) | col))


def _top24(w):
    return (w >> _U64(40)).astype(_F32) * _F32(1.0 / 16777216.0)


def _mid24(w):
    return ((w >> _U64(16)) & _U64(0xFFFFFF)).astype(_F32) * _F32(1.0 / 16777216.0)


def gaps_numpy(seed: int, n_sites: int, bp_per_site: float) -> np.ndarray:
    """Site spacings: 1 for the first site, else max(1, floor(-ln(1-u) bp))."""
    s = np.arange(n_sites, dtype=_U64)
    u = (_draw(_key(seed, 15), 0, s) >> _U64(11)).astype(np.float64) * 2.0 ** -53
    g = np.maximum(np.floor(-np.log1p(-u) * float(bp_per_site)), 1.0).astype(np.int64)
    if n_sites:
        g[0] = 1
    return g


def site_p_numpy(seed: int, tag: int, n_sites: int):
    """(x^2, x^2 + y^2) per site for (x, y) uniform in the unit disk; the
    site frequency is their ratio, arcsine distributed."""
    kp = _key(seed, tag)
    xx = np.full(n_sites, 0.5, dtype=_F32)
    r = np.ones(n_sites, dtype=_F32)
    todo = np.arange(n_sites, dtype=_U64)
    for t in range(64):
        if todo.size == 0:
            break
        x = _F32(2.0) * _top24(_draw(kp, 2 * t, todo)) - _F32(1.0)
        y = _F32(2.0) * _top24(_draw(kp, 2 * t + 1, todo)) - _F32(1.0)
        x2 = x * x
        rr = x2 + y * y
        ok = (rr <= _F32(1.0)) & (rr > _F32(0.0))
        idx = todo[ok].astype(np.int64)
        xx[idx] = x2[ok]
        r[idx] = rr[ok]
        todo = todo[~ok]
    return xx, r


def founders_numpy(seed: int, tag: int, n_founders: int, n_sites: int,
                   base: Optional[np.ndarray] = None, share: float = 0.0) -> np.ndarray:
    """Founder alleles [F][M]: derived when u (x^2 + y^2) < x^2; with base,
    each entry is base's with probability share."""
    xx, r = site_p_numpy(seed, tag, n_sites)
    f = np.arange(n_founders, dtype=_U64)[:, None]
    s = np.arange(n_sites, dtype=_U64)[None, :]
    out = ((_top24(_draw(_key(seed, tag + 1), f, s)) * r[None, :]) < xx[None, :]).astype(np.uint8)
    if base is not None:
        keep = _top24(_draw(_key(seed, tag + 2), f, s)) < _F32(share)
        out = np.where(keep, base, out).astype(np.uint8)
    return out


def copy_numpy(seed: int, tag: int, founders: np.ndarray, n_haps: int, switch_p: float,
               flip_p: float) -> np.ndarray:
    """Alleles [M][n] copied from the founders along each haplotype's path."""
    F, M = founders.shape
    h = np.arange(n_haps, dtype=_U64)
    w = _draw(_key(seed, tag + 3), h[:, None], np.arange(M, dtype=_U64)[None, :])
    switch = _top24(w) < _F32(switch_p)
    switch[:, 0] = False
    off = np.where(switch, 1 + (((_U64(F - 1) * (w & _U64(0xFFFF))) >> _U64(16)).astype(np.int64)), 0)
    f0 = ((_draw(_key(seed, tag + 5), h, 0) >> _U64(32)) * _U64(F)) >> _U64(32)
    path = (f0.astype(np.int64)[:, None] + np.cumsum(off, axis=1)) % F
    a = founders[path, np.arange(M)[None, :]]
    a ^= (_mid24(w) < _F32(flip_p)).astype(np.uint8)
    return np.ascontiguousarray(a.T)


def region_numpy(spec: "RequestSpec"):
    """The served request's inputs on the host: (alleles_a, alleles_b or None,
    pos_bp, gpos_cm), equal to device_region's."""
    c = SERVE
    F, M = c["n_founders"], spec.n_sites
    pos = np.cumsum(gaps_numpy(spec.seed, M, c["bp_per_site"]))
    fa = founders_numpy(spec.seed, 0, F, M)
    a = copy_numpy(spec.seed, 0, fa, spec.n_a, c["switch_p"], c["flip_p"])
    b = None
    if spec.kind == "xpehh":
        fb = founders_numpy(spec.seed, 8, F, M, fa, c["share_p"])
        b = copy_numpy(spec.seed, 8, fb, spec.n_b, c["switch_p"], c["flip_p"])
    return a, b, pos, pos.astype(np.float64) * 1e-6


def build_gpu(arch: str = "gfx950") -> str:
    """Compile gen.hip into libhapgen_gpu.so (always recompiles)."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = GEN_LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=" + arch, "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(HERE, "gen.hip"), "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    os.replace(tmp, GEN_LIB)
    return GEN_LIB


_GEN = None


def _gen_lib():
    global _GEN
    if _GEN is None:
        import ctypes as C
        if not os.path.exists(GEN_LIB):
            raise RuntimeError("%s is not built (hapgen.build_gpu())" % GEN_LIB)
        lib = C.CDLL(GEN_LIB)
        p, i64, u64, i32, f32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_int, C.c_float
        lib.hg_gaps.argtypes = [u64, i64, C.c_double, p, p]
        lib.hg_founders.argtypes = [u64, i32, i32, i64, p, f32, p, p]
        lib.hg_block_offsets.argtypes = [u64, i32, i32, i64, i32, f32, p, p]
        lib.hg_copy.argtypes = [u64, i32, p, i32, i64, i32, f32, f32, p, p, p]
        for f in (lib.hg_gaps, lib.hg_founders, lib.hg_block_offsets, lib.hg_copy):
            f.restype = C.c_int
        _GEN = lib
    return _GEN


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError("%s failed (%d)" % (what, rc))


def _copy_device(lib, stream, seed: int, tag: int, founders, n_haps: int, switch_p: float,
                 flip_p: float):
    import torch
    F, M = founders.shape
    dev = founders.device
    out = torch.empty((M, n_haps), dtype=torch.uint8, device=dev)
    if n_haps == 0:
        return out
    nb = (M + 63) // 64
    sums = torch.empty((n_haps, nb), dtype=torch.int32, device=dev)
    _check(lib.hg_block_offsets(seed, tag, F, M, n_haps, switch_p, sums.data_ptr(), stream),
           "hg_block_offsets")
    excl = torch.cumsum(sums, dim=1, dtype=torch.int64) - sums
    _check(lib.hg_copy(seed, tag, founders.data_ptr(), F, M, n_haps, switch_p, flip_p,
                       excl.data_ptr(), out.data_ptr(), stream), "hg_copy")
    return out


def device_region(spec: RequestSpec, device="cuda"):
    """Inputs of one served request, generated on the GPU ``device`` from its
    seed on the current stream: (alleles_a, alleles_b or None, pos_bp,
    gpos_cm) as torch tensors, equal to region_numpy's.

    Positions: a Poisson process of about one site per bp_per_site bp
    (exponential spacings, each at least 1 bp) starting at 1; 1 cM/Mb."""
    import torch
    c = SERVE
    lib = _gen_lib()
    dev = torch.device(device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    F, M, seed = c["n_founders"], spec.n_sites, int(spec.seed)
    gaps = torch.empty(M, dtype=torch.int64, device=dev)
    _check(lib.hg_gaps(seed, M, float(c["bp_per_site"]), gaps.data_ptr(), stream), "hg_gaps")
    pos = torch.cumsum(gaps, 0)
    gpos = pos.to(torch.float64) * 1e-6
    fa = torch.empty((F, M), dtype=torch.uint8, device=dev)
    _check(lib.hg_founders(seed, 0, F, M, None, 0.0, fa.data_ptr(), stream), "hg_founders")
    a = _copy_device(lib, stream, seed, 0, fa, spec.n_a, c["switch_p"], c["flip_p"])
    b = None
    if spec.kind == "xpehh":
        fb = torch.empty((F, M), dtype=torch.uint8, device=dev)
        _check(lib.hg_founders(seed, 8, F, M, fa.data_ptr(), c["share_p"], fb.data_ptr(), stream),
               "hg_founders")
        b = _copy_device(lib, stream, seed, 8, fb, spec.n_b, c["switch_p"], c["flip_p"])
    return (a, b, pos, gpos)
