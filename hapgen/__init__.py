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
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "HapData", "draw_positions", "draw_founders", "derive_founders",
    "copy_haplotypes", "plant_sweep", "copying_model", "config_input",
    "random_haplotypes", "CONFIGS", "CopyEvents", "draw_copy_events", "render_alleles",
    "plant_sweep_tensor", "large_batch_input", "poisson_arrivals", "log_uniform_int",
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
# device from per-request seeds (torch's counter-based generator), so that a
# request stream of ~10^11 alleles does not wait on the host.
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


def _device_copy(gen, founders, n_haps: int, switch_p: float, flip_p: float, chunk: int = 16384):
    """Founder copying on the device, drawn haplotype-major so that the
    founder path is a scan along the contiguous axis; returned site-major.

    One uniform u per (haplotype, site) decides the switch (u < switch_p) and,
    rescaled to [0, 1), which other founder is taken next; a second uniform
    decides the flip."""
    import torch
    F, M = founders.shape
    dev = founders.device
    out = torch.empty((M, n_haps), dtype=torch.uint8, device=dev)
    cur = torch.randint(0, F, (n_haps,), generator=gen, device=dev).to(torch.int32)
    for s0 in range(0, M, chunk):
        s1 = min(M, s0 + chunk)
        u = torch.rand((n_haps, s1 - s0), generator=gen, device=dev)
        if F >= 2:
            step = torch.where(u < switch_p,
                               1 + torch.clamp((u * (1.0 / switch_p) * (F - 1)).to(torch.int32),
                                               max=F - 2),
                               torch.zeros((), dtype=torch.int32, device=dev))
        else:
            step = torch.zeros_like(u, dtype=torch.int32)
        if s0 == 0:
            step[:, 0] = 0
        path = torch.remainder(cur[:, None] + torch.cumsum(step, dim=1, dtype=torch.int32), F)
        cur = path[:, -1].clone()
        col = torch.arange(s0, s1, device=dev, dtype=torch.int32)[None, :]
        block = founders[path.long(), col.long()]
        flips = torch.rand((n_haps, s1 - s0), generator=gen, device=dev) < flip_p
        out[s0:s1] = (block ^ flips.to(torch.uint8)).t()
    return out


def device_region(spec: RequestSpec, device="cuda"):
    """Inputs of one served request, generated on ``device``: (alleles_a,
    alleles_b or None, pos_bp, gpos_cm) as torch tensors; positions are drawn
    on the host from the same seed."""
    import torch
    c = SERVE
    rng = np.random.default_rng(spec.seed)
    pos, gpos = draw_positions(rng, spec.n_sites, max(spec.n_sites, spec.n_sites * c["bp_per_site"]))
    gen = torch.Generator(device=device)
    gen.manual_seed(int(spec.seed))
    F, M = c["n_founders"], spec.n_sites
    # Beta(1/2, 1/2) is the arcsine law: sin^2(pi U / 2)
    p = torch.sin(0.5 * math.pi * torch.rand(M, generator=gen, device=device)) ** 2
    fa = (torch.rand((F, M), generator=gen, device=device) < p[None, :]).to(torch.uint8)
    a = _device_copy(gen, fa, spec.n_a, c["switch_p"], c["flip_p"])
    b = None
    if spec.kind == "xpehh":
        p2 = torch.sin(0.5 * math.pi * torch.rand(M, generator=gen, device=device)) ** 2
        fresh = (torch.rand((F, M), generator=gen, device=device) < p2[None, :]).to(torch.uint8)
        keep = torch.rand((F, M), generator=gen, device=device) < c["share_p"]
        fb = torch.where(keep, fa, fresh)
        b = _device_copy(gen, fb, spec.n_b, c["switch_p"], c["flip_p"])
    return (a, b, torch.from_numpy(pos).to(device), torch.from_numpy(gpos).to(device))
