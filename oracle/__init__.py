"""Plain FP64 CPU oracle for EHH / iHS / XPEHH (test infrastructure only).

The arithmetic lives in ``selscan_oracle.c`` (plain C, built with gcc
``-O2 -ffp-contract=off -fopenmp``); this module only loads it with ctypes and
marshals numpy arrays.  Nothing in the product package may import this module:
it exists so that the tests, the smoke check and the benchmark's CPU-baseline
leg can check and time the GPU library against the paper's definitions.

Inputs are plain site-major 0/1 allele matrices ``uint8[n_sites, n_haps]``
(0 ancestral, 1 derived), physical positions ``int64[n_sites]`` and genetic
positions ``float64[n_sites]`` in cM.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "selscan_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {"OK": 0, "MAF": 1, "EDGE": 2, "GAP": 3, "UNDEFINED": 4, "BIN": 5, "CAPACITY": 6}


@dataclasses.dataclass
class Params:
    """The paper's flexible parameters (Sec. 1.2, Sec. 1.3) with its defaults."""
    ehh_cutoff: float = 0.05
    maf_cutoff: float = 0.05
    gap_scale_bp: int = 20_000
    max_gap_bp: int = 200_000
    bin_width: float = 0.025
    physical_map: int = 0      # 1: integrate over physical distance (bp)


class _CParams(ctypes.Structure):
    _fields_ = [("ehh_cutoff", ctypes.c_double), ("maf_cutoff", ctypes.c_double),
                ("gap_scale_bp", ctypes.c_int64), ("max_gap_bp", ctypes.c_int64),
                ("bin_width", ctypes.c_double), ("physical_map", ctypes.c_int32)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("SS_ORACLE_LIB", _LIB)   # tests swap in planted mistakes
        if path == _LIB and not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.or_ihs.argtypes = [P, i64, i64, P, P, ctypes.POINTER(_CParams), P, i64,
                               P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.or_xpehh.argtypes = [P, i64, P, i64, i64, P, P, ctypes.POINTER(_CParams), P, i64,
                                 P, P, P, P, P, P, ctypes.c_int]
        lib.or_ehh.argtypes = [P, i64, i64, P, P, ctypes.POINTER(_CParams), i64, i64,
                               P, P, P, P, P, P]
        lib.or_xpehh_trace.argtypes = [P, i64, P, i64, i64, P, P, ctypes.POINTER(_CParams),
                                       i64, i64, P, P, P, P]
        lib.or_standardize.argtypes = [P, P, P, i64, ctypes.c_int, P, P, P, P]
        for f in (lib.or_ihs, lib.or_xpehh, lib.or_ehh, lib.or_xpehh_trace, lib.or_standardize):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _cp(p: Params) -> _CParams:
    return _CParams(float(p.ehh_cutoff), float(p.maf_cutoff), int(p.gap_scale_bp),
                    int(p.max_gap_bp), float(p.bin_width), int(p.physical_map))


def _prep(alleles, pos, gpos):
    H = np.ascontiguousarray(alleles, dtype=np.uint8)
    pos = np.ascontiguousarray(pos, dtype=np.int64)
    gpos = np.ascontiguousarray(gpos, dtype=np.float64)
    if H.ndim != 2 or pos.shape[0] != H.shape[0] or gpos.shape[0] != H.shape[0]:
        raise ValueError("alleles must be [n_sites, n_haps] with matching positions")
    return H, pos, gpos


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def ihs(alleles, pos, gpos, params: Params = Params(), loci=None, threads: int = 0):
    """iHS scan (Sec. 1.2).  ``loci`` restricts the scan to a list of sites
    (standardization is then skipped).  Returns a dict of numpy arrays."""
    H, pos, gpos = _prep(alleles, pos, gpos)
    M, n = H.shape
    out = {k: np.full(M, np.nan) for k in ("ihh1", "ihh0", "unstd", "std", "freq")}
    out["status"] = np.full(M, -1, dtype=np.int8)
    out["bin"] = np.full(M, -1, dtype=np.int32)
    out["steps"] = np.zeros((M, 2, 2), dtype=np.int64)
    lo = None
    nl = 0
    if loci is not None:
        lo = np.ascontiguousarray(loci, dtype=np.int64)
        nl = lo.shape[0]
    cp = _cp(params)
    rc = _load().or_ihs(_ptr(H), n, M, _ptr(pos), _ptr(gpos), ctypes.byref(cp), _ptr(lo), nl,
                        _ptr(out["ihh1"]), _ptr(out["ihh0"]), _ptr(out["unstd"]),
                        _ptr(out["std"]), _ptr(out["freq"]), _ptr(out["status"]),
                        _ptr(out["bin"]), _ptr(out["steps"]), int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("oracle or_ihs failed (%d)" % rc)
    return out


def xpehh(alleles_a, alleles_b, pos, gpos, params: Params = Params(), loci=None,
          threads: int = 0):
    """XPEHH scan (Sec. 1.3) of population A against B on the same sites."""
    A, pos, gpos = _prep(alleles_a, pos, gpos)
    B = np.ascontiguousarray(alleles_b, dtype=np.uint8)
    if B.ndim != 2 or B.shape[0] != A.shape[0]:
        raise ValueError("populations must share their sites")
    M, nA = A.shape
    nB = B.shape[1]
    out = {k: np.full(M, np.nan) for k in ("ihhA", "ihhB", "unstd", "std")}
    out["status"] = np.full(M, -1, dtype=np.int8)
    out["steps"] = np.zeros((M, 2), dtype=np.int64)
    lo = None
    nl = 0
    if loci is not None:
        lo = np.ascontiguousarray(loci, dtype=np.int64)
        nl = lo.shape[0]
    cp = _cp(params)
    rc = _load().or_xpehh(_ptr(A), nA, _ptr(B), nB, M, _ptr(pos), _ptr(gpos), ctypes.byref(cp),
                          _ptr(lo), nl, _ptr(out["ihhA"]), _ptr(out["ihhB"]), _ptr(out["unstd"]),
                          _ptr(out["std"]), _ptr(out["status"]), _ptr(out["steps"]),
                          int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("oracle or_xpehh failed (%d)" % rc)
    return out


def ehh(alleles, pos, gpos, core: int, params: Params = Params(), cap: int = 4096,
        sizes: bool = False):
    """EHH curves at one core site (Sec. 1.1, Eqs. 1 and 3), both directions.

    Returns S [2 dirs, cap+1, 2] (S_0, S_1 = sum over each core's classes of
    C(n_h,2)), ehh [2, cap+1, 3] (EHH_0, EHH_1, whole-sample EHH), len [2],
    optionally class sizes [2, cap+1, n] (core in bit 31), ihh [2]
    (iHH_0, iHH_1) and the status.
    """
    H, pos, gpos = _prep(alleles, pos, gpos)
    M, n = H.shape
    S = np.zeros((2, cap + 1, 2), dtype=np.uint64)
    E = np.zeros((2, cap + 1, 3), dtype=np.float64)
    L = np.zeros(2, dtype=np.int64)
    Z = np.zeros((2, cap + 1, n), dtype=np.uint32) if sizes else None
    ihh_ = np.zeros(2, dtype=np.float64)
    st = np.zeros(1, dtype=np.int8)
    cp = _cp(params)
    rc = _load().or_ehh(_ptr(H), n, M, _ptr(pos), _ptr(gpos), ctypes.byref(cp), int(core), int(cap),
                        _ptr(S), _ptr(E), _ptr(L), _ptr(Z), _ptr(ihh_), _ptr(st))
    if rc != 0:
        raise RuntimeError("oracle or_ehh failed (%d)" % rc)
    return {"S": S, "ehh": E, "len": L, "sizes": Z, "ihh": ihh_, "status": int(st[0])}


def xpehh_trace(alleles_a, alleles_b, pos, gpos, site: int, params: Params = Params(),
                cap: int = 4096):
    """Per-marker S_A, S_B, S_pool of the pooled XPEHH walk at one site."""
    A, pos, gpos = _prep(alleles_a, pos, gpos)
    B = np.ascontiguousarray(alleles_b, dtype=np.uint8)
    M, nA = A.shape
    nB = B.shape[1]
    S = np.zeros((2, cap + 1, 3), dtype=np.uint64)
    L = np.zeros(2, dtype=np.int64)
    ihh_ = np.zeros(2, dtype=np.float64)
    st = np.zeros(1, dtype=np.int8)
    cp = _cp(params)
    rc = _load().or_xpehh_trace(_ptr(A), nA, _ptr(B), nB, M, _ptr(pos), _ptr(gpos),
                                ctypes.byref(cp), int(site), int(cap), _ptr(S), _ptr(L),
                                _ptr(ihh_), _ptr(st))
    if rc != 0:
        raise RuntimeError("oracle or_xpehh_trace failed (%d)" % rc)
    return {"S": S, "len": L, "ihh": ihh_, "status": int(st[0])}


def standardize(u, status, bins, nbins: int):
    """Frequency-bin standardization (Eq. 6; Eq. 9 with one bin)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    st = np.array(status, dtype=np.int8, copy=True)
    b = np.ascontiguousarray(bins, dtype=np.int32)
    M = u.shape[0]
    z = np.full(M, np.nan)
    mean = np.zeros(nbins)
    sd = np.zeros(nbins)
    cnt = np.zeros(nbins, dtype=np.int64)
    _load().or_standardize(_ptr(u), _ptr(st), _ptr(b), M, int(nbins), _ptr(z), _ptr(mean),
                           _ptr(sd), _ptr(cnt))
    return {"std": z, "status": st, "mean": mean, "sd": sd, "n": cnt}


def genome_standardize(outs, nbins: int):
    """Standardization over the whole genome (Eq. 6 for iHS with ``nbins``
    frequency bins, Eq. 9 for XPEHH with one): the scored loci (status OK or
    BIN) of several scans, concatenated in list order and site order, go
    through ``or_standardize`` together.  ``outs`` are oracle scan outputs
    (iHS scans carry their ``bin``).  Returns one {"std", "status"} per scan
    and the bin statistics {"mean", "sd", "n"}."""
    u = np.concatenate([np.asarray(o["unstd"], dtype=np.float64) for o in outs])
    st = np.concatenate([np.where(np.asarray(o["status"]) == STATUS["BIN"], STATUS["OK"],
                                  np.asarray(o["status"])).astype(np.int8) for o in outs])
    b = np.concatenate([np.asarray(o["bin"], dtype=np.int32) if nbins > 1
                        else np.zeros(len(o["unstd"]), dtype=np.int32) for o in outs])
    r = standardize(u, st, b, nbins)
    res, at = [], 0
    for o in outs:
        m = len(o["unstd"])
        res.append({"std": r["std"][at:at + m], "status": r["status"][at:at + m]})
        at += m
    return res, {"mean": r["mean"], "sd": r["sd"], "n": r["n"]}
