"""Brute-force pair enumeration for tiny inputs (test infrastructure only).

Independent of ``selscan_oracle.c``: instead of refining a partition, it uses
the identity behind Eq. 1 and Eq. 3 of the paper (Sec. 1.1) that
sum_h C(n_h, 2) over the distinct haplotypes on [x0, x_i] equals the number
of unordered pairs of haplotypes that are identical at every marker from x0
out to x_i.  Pure Python loops: only for n and walk lengths in the tens.
"""
from __future__ import annotations

import itertools


def identical_pairs(alleles, core: int, step: int, direction: int, hap_subset=None):
    """Number of unordered haplotype pairs identical on the markers
    core, core+direction, ..., core+direction*step."""
    n = len(alleles[0])
    haps = range(n) if hap_subset is None else hap_subset
    sites = [core + direction * t for t in range(step + 1)]
    count = 0
    for a, b in itertools.combinations(haps, 2):
        if all(alleles[s][a] == alleles[s][b] for s in sites):
            count += 1
    return count


def core_sums(alleles, core: int, step: int, direction: int):
    """(S_0, S_1): identical pairs among the carriers of allele 0 / 1 at x0."""
    n = len(alleles[0])
    c0 = [h for h in range(n) if alleles[core][h] == 0]
    c1 = [h for h in range(n) if alleles[core][h] == 1]
    return (identical_pairs(alleles, core, step, direction, c0),
            identical_pairs(alleles, core, step, direction, c1))


def pooled_sums(alleles_a, alleles_b, core: int, step: int, direction: int):
    """(S_A, S_B, S_pool) for the pooled walk of two populations."""
    nA = len(alleles_a[0])
    pooled = [list(ra) + list(rb) for ra, rb in zip(alleles_a, alleles_b)]
    n = len(pooled[0])
    sa = identical_pairs(pooled, core, step, direction, range(nA))
    sb = identical_pairs(pooled, core, step, direction, range(nA, n))
    sp = identical_pairs(pooled, core, step, direction, range(n))
    return sa, sb, sp


def class_sizes(alleles, core: int, step: int, direction: int):
    """Sorted multiset of (core allele, class size) for classes of size >= 2,
    obtained by grouping the haplotype strings themselves."""
    n = len(alleles[0])
    sites = [core + direction * t for t in range(step + 1)]
    groups = {}
    for h in range(n):
        key = tuple(alleles[s][h] for s in sites)
        groups[key] = groups.get(key, 0) + 1
    return sorted((key[0], c) for key, c in groups.items() if c >= 2)
