"""MI355X-native EHH / iHS / XPEHH scans (Szpiech & Hernandez, arXiv:1403.6854).

Thin Python binding over the C ABI of ``libselscan_hip.so``
(``include/selscan_hip.h``): argument marshalling only.  Every step of the
scans runs in the library's HIP kernels; PyTorch provides device memory and
streams.  There is no CPU fallback: if the library is not built, importing the
entry points raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libselscan_hip.so")

SS_OK, SS_EARG, SS_ESHAPE, SS_EWS, SS_EDEV = 0, -1, -2, -3, -4
OP_EHH, OP_IHS, OP_XPEHH = 0, 1, 2
STATUS_NAMES = {0: "OK", 1: "MAF", 2: "EDGE", 3: "GAP", 4: "UNDEFINED", 5: "BIN", 6: "CAPACITY"}


class SelscanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("selscan_hip error %d: %s" % (code, msg))
        self.code = code


@dataclasses.dataclass
class Params:
    """Flexible parameters of Sec. 1.2 / 1.3, with the paper's defaults."""
    ehh_cutoff: float = 0.05
    maf_cutoff: float = 0.05
    gap_scale_bp: int = 20_000
    max_gap_bp: int = 200_000
    bin_width: float = 0.025
    physical_map: int = 0      # 1: integrate over pos_bp (g in bp) instead of gpos_cm


class _Params(ctypes.Structure):
    _fields_ = [("ehh_cutoff", ctypes.c_double), ("maf_cutoff", ctypes.c_double),
                ("gap_scale_bp", ctypes.c_int64), ("max_gap_bp", ctypes.c_int64),
                ("bin_width", ctypes.c_double), ("physical_map", ctypes.c_int32)]


class _HapMat(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("n_haps", ctypes.c_int64),
                ("n_sites", ctypes.c_int64), ("words_per_site", ctypes.c_int64),
                ("pos_bp", ctypes.c_void_p), ("gpos_cm", ctypes.c_void_p)]


class _Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("a", _HapMat), ("b", _HapMat),
                ("d_ihh_x", ctypes.c_void_p), ("d_ihh_y", ctypes.c_void_p),
                ("d_unstd", ctypes.c_void_p), ("d_std", ctypes.c_void_p),
                ("d_freq", ctypes.c_void_p), ("d_status", ctypes.c_void_p),
                ("d_steps", ctypes.c_void_p)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("pair_cap", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32), ("small_kernel", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("small_pair_cap", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("class_cap", ctypes.c_int32),
                ("counter_copies", ctypes.c_int32)]


class _StdRegion(ctypes.Structure):
    _fields_ = [("d_unstd", ctypes.c_void_p), ("d_freq", ctypes.c_void_p),
                ("d_status", ctypes.c_void_p), ("d_std", ctypes.c_void_p),
                ("n_sites", ctypes.c_int64), ("n_haps", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libselscan_hip.so is not built; run paper_1403_6854_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
        HM = ctypes.POINTER(_HapMat)
        PR = ctypes.POINTER(_Params)
        L.ss_version.restype = ctypes.c_char_p
        L.ss_last_error.restype = ctypes.c_char_p
        L.ss_default_params.argtypes = [PR]
        L.ss_pack.argtypes = [P, i64, i64, i64, P, P]
        L.ss_workspace_bytes.argtypes = [ctypes.c_int, HM, HM, PR, i64]
        L.ss_workspace_bytes.restype = sz
        L.ss_ehh.argtypes = [HM, i64, PR, i64, P, P, P, P, P, P, P, sz, P]
        L.ss_ihs.argtypes = [HM, PR, P, P, P, P, P, P, P, P, sz, P]
        L.ss_xpehh.argtypes = [HM, HM, PR, P, P, P, P, P, P, P, sz, P]
        L.ss_ihs_static.argtypes = [HM, PR, P, P, P, P, P, P, P, P]
        L.ss_static_scratch_bytes.argtypes = []
        L.ss_static_scratch_bytes.restype = sz
        D = ctypes.POINTER(ctypes.c_double)
        L.ss_micro_out_words.argtypes = []
        L.ss_micro_copy.argtypes = [P, P, sz, ctypes.c_int, P, D]
        L.ss_micro_valu.argtypes = [P, ctypes.c_int, ctypes.c_int, P, D, D]
        L.ss_micro_lds_atomic.argtypes = [P, ctypes.c_int, ctypes.c_int, P, D, D]
        L.ss_micro_cell.argtypes = [P, i64, P, ctypes.c_int, ctypes.c_int, P, D, D]
        for f in ("ss_micro_out_words", "ss_micro_copy", "ss_micro_valu", "ss_micro_lds_atomic",
                  "ss_micro_cell"):
            getattr(L, f).restype = ctypes.c_int
        SR = ctypes.POINTER(_StdRegion)
        L.ss_genome_workspace_bytes.argtypes = [SR, ctypes.c_int32, ctypes.c_int32, PR]
        L.ss_genome_workspace_bytes.restype = sz
        L.ss_genome_standardize.argtypes = [SR, ctypes.c_int32, ctypes.c_int32, PR, P, P, sz, P]
        L.ss_set_walk_kernel.argtypes = [ctypes.c_int]
        L.ss_set_mask_lanes.argtypes = [ctypes.c_int]
        L.ss_set_mask_skip.argtypes = [ctypes.c_int]
        L.ss_timing_enable.argtypes = [ctypes.c_int]
        L.ss_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_int]
        RQ = ctypes.POINTER(_Request)
        BC = ctypes.POINTER(_BatchConfig)
        L.ss_batch_workspace_bytes.argtypes = [RQ, ctypes.c_int32, PR]
        L.ss_batch_workspace_bytes.restype = sz
        L.ss_scan_batch.argtypes = [RQ, ctypes.c_int32, PR, P, sz, P]
        L.ss_get_batch_config.argtypes = [BC]
        L.ss_set_batch_config.argtypes = [BC]
        L.ss_autotune_batch.argtypes = [RQ, ctypes.c_int32, PR, P, sz, P, i64, BC,
                                        ctypes.POINTER(ctypes.c_double)]
        L.ss_set_graph.argtypes = [ctypes.c_int]
        L.ss_graph_clear.argtypes = []
        L.ss_set_group_tuning.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
        L.ss_get_group_tuning.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]
        for f in ("ss_pack", "ss_ehh", "ss_ihs", "ss_ihs_static", "ss_genome_standardize", "ss_xpehh", "ss_set_walk_kernel", "ss_set_mask_lanes", "ss_set_mask_skip",
                  "ss_timing_enable", "ss_timing_read", "ss_scan_batch", "ss_get_batch_config",
                  "ss_set_batch_config", "ss_autotune_batch", "ss_set_graph", "ss_graph_clear",
                  "ss_get_group_tuning", "ss_set_group_tuning"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SS_OK:
        raise SelscanError(rc, lib().ss_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _cparams(p: Optional[Params]) -> _Params:
    p = p or Params()
    return _Params(float(p.ehh_cutoff), float(p.maf_cutoff), int(p.gap_scale_bp),
                   int(p.max_gap_bp), float(p.bin_width), int(p.physical_map))


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU")


@dataclasses.dataclass
class HapMat:
    """A bit-packed marker-major haplotype matrix resident on the device.

    bits: int64 [n_sites, words_per_site] (uint64 words; haplotype h is bit
    h % 64 of word h // 64; 1 = derived allele); pos_bp: int64 [n_sites];
    gpos_cm: float64 [n_sites].
    """
    bits: torch.Tensor
    n_haps: int
    pos_bp: torch.Tensor
    gpos_cm: torch.Tensor

    @property
    def n_sites(self) -> int:
        return int(self.bits.shape[0])

    @property
    def words_per_site(self) -> int:
        return int(self.bits.stride(0))

    def desc(self) -> _HapMat:
        if self.bits.dtype != torch.int64 or self.bits.dim() != 2 or self.bits.stride(1) != 1:
            raise ValueError("bits must be a row-contiguous int64 [n_sites, words] tensor")
        if self.pos_bp.dtype != torch.int64 or self.gpos_cm.dtype != torch.float64:
            raise ValueError("pos_bp must be int64 and gpos_cm float64")
        if not (self.pos_bp.is_contiguous() and self.gpos_cm.is_contiguous()):
            raise ValueError("position arrays must be contiguous")
        if self.pos_bp.numel() != self.n_sites or self.gpos_cm.numel() != self.n_sites:
            raise ValueError("position arrays must have n_sites entries")
        _need_cuda(self.bits, self.pos_bp, self.gpos_cm)
        return _HapMat(self.bits.data_ptr(), int(self.n_haps), self.n_sites, self.words_per_site,
                       self.pos_bp.data_ptr(), self.gpos_cm.data_ptr())

    def validate(self):
        """Content checks the C ABI leaves to the caller: sorted positions and
        zero padding bits (one device round trip)."""
        bad = torch.zeros((), dtype=torch.bool, device=self.bits.device)
        if self.n_sites > 1:
            bad |= (self.pos_bp[1:] < self.pos_bp[:-1]).any()
            bad |= (self.gpos_cm[1:] < self.gpos_cm[:-1]).any()
        words = (self.n_haps + 63) // 64
        rem = self.n_haps - 64 * (words - 1)
        if rem < 64:
            mask = ~((1 << rem) - 1)
            mask = mask if mask >= -(1 << 63) else mask + (1 << 64)
            bad |= (self.bits[:, words - 1] & mask).ne(0).any()
        if self.words_per_site > words:
            bad |= self.bits[:, words:].ne(0).any()
        if bool(bad):
            raise ValueError("positions must be non-decreasing and padding bits zero")


def words_for(n_haps: int) -> int:
    return (int(n_haps) + 63) // 64


def pack(alleles: torch.Tensor, stream=None) -> torch.Tensor:
    """Bit-pack a uint8 [n_sites, n_haps] 0/1 matrix on the device."""
    _need_cuda(alleles)
    if alleles.dtype != torch.uint8 or alleles.dim() != 2:
        raise ValueError("alleles must be uint8 [n_sites, n_haps]")
    alleles = alleles.contiguous()
    M, n = alleles.shape
    W = words_for(n)
    bits = torch.empty((M, W), dtype=torch.int64, device=alleles.device)
    _check(lib().ss_pack(_ptr(alleles), n, M, W, _ptr(bits), _stream(stream)))
    return bits


def hapmat(alleles: torch.Tensor, pos_bp: torch.Tensor, gpos_cm: torch.Tensor,
           stream=None) -> HapMat:
    """Pack device-resident alleles into a HapMat."""
    return HapMat(pack(alleles, stream), int(alleles.shape[1]), pos_bp.contiguous(),
                  gpos_cm.contiguous())


def workspace_bytes(op: int, a: HapMat, b: Optional[HapMat] = None,
                    params: Optional[Params] = None, ehh_cap: int = 0) -> int:
    da = a.desc()
    db = b.desc() if b is not None else None
    cp = _cparams(params)
    n = lib().ss_workspace_bytes(op, ctypes.byref(da), ctypes.byref(db) if db else None,
                                 ctypes.byref(cp), int(ehh_cap))
    if n == 0:
        raise SelscanError(SS_EARG, "invalid arguments for ss_workspace_bytes")
    return int(n)


def _workspace(nbytes: int, device, ws: Optional[torch.Tensor]):
    if ws is not None and ws.numel() * ws.element_size() >= nbytes:
        return ws
    return torch.empty(nbytes + 256, dtype=torch.uint8, device=device)


def _aligned(ws: torch.Tensor) -> int:
    p = ws.data_ptr()
    return (p + 255) & ~255


def ihs(h: HapMat, params: Optional[Params] = None, steps: bool = False, stream=None,
        ws: Optional[torch.Tensor] = None, out: Optional[dict] = None, validate: bool = True):
    """iHS scan over every site (Sec. 1.2).  Returns a dict of device tensors:
    ihh1, ihh0, unstd, std, freq (float64), status (int8) and optionally
    steps (int32 [n_sites, 2, 2])."""
    if validate:
        h.validate()
    d = h.desc()
    M = h.n_sites
    dev = h.bits.device
    nb = workspace_bytes(OP_IHS, h, None, params)
    ws = _workspace(nb, dev, ws)
    if out is None:
        out = {k: torch.empty(M, dtype=torch.float64, device=dev)
               for k in ("ihh1", "ihh0", "unstd", "std", "freq")}
        out["status"] = torch.empty(M, dtype=torch.int8, device=dev)
        if steps:
            out["steps"] = torch.empty((M, 2, 2), dtype=torch.int32, device=dev)
    cp = _cparams(params)
    base = _aligned(ws)
    avail = ws.numel() - (base - ws.data_ptr())
    _check(lib().ss_ihs(ctypes.byref(d), ctypes.byref(cp), _ptr(out["ihh1"]), _ptr(out["ihh0"]),
                        _ptr(out["unstd"]), _ptr(out["std"]), _ptr(out["freq"]),
                        _ptr(out["status"]), _ptr(out.get("steps")), ctypes.c_void_p(base),
                        avail, _stream(stream)))
    return out


def ihs_static(h: HapMat, params: Optional[Params] = None, steps: bool = False, stream=None,
               out: Optional[dict] = None, validate: bool = True):
    """The iHS scan of ``ihs`` through ss_ihs_static: no workspace, the
    library's static device scratch instead (scans up to
    ``static_scratch_bytes()`` of scratch).  Pass ``out`` to allocate nothing
    here either."""
    if validate:
        h.validate()
    d = h.desc()
    M = h.n_sites
    dev = h.bits.device
    if out is None:
        out = {k: torch.empty(M, dtype=torch.float64, device=dev)
               for k in ("ihh1", "ihh0", "unstd", "std", "freq")}
        out["status"] = torch.empty(M, dtype=torch.int8, device=dev)
        if steps:
            out["steps"] = torch.empty((M, 2, 2), dtype=torch.int32, device=dev)
    cp = _cparams(params)
    _check(lib().ss_ihs_static(ctypes.byref(d), ctypes.byref(cp), _ptr(out["ihh1"]),
                               _ptr(out["ihh0"]), _ptr(out["unstd"]), _ptr(out["std"]),
                               _ptr(out["freq"]), _ptr(out["status"]), _ptr(out.get("steps")),
                               _stream(stream)))
    return out


def genome_standardize(outs: Sequence[dict], n_haps: Optional[Sequence[int]] = None,
                       op: int = OP_IHS, params: Optional[Params] = None, stream=None,
                       ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Standardize the scores of many scans together (Sec. 1.2 Eq. 6 and
    Sec. 1.3 Eq. 9 over the whole genome), in place: ``outs`` are the output
    dicts of ``ihs`` / ``xpehh`` / batch requests (their ``unstd``, ``freq``,
    ``status`` and ``std``), taken as one sequence of loci in list order;
    ``n_haps`` gives each iHS scan's haplotype count (its bins come from
    ``freq``).  Returns the per-bin statistics [nbins, 3] = N, mean, SD."""
    if not outs:
        raise ValueError("no scans")
    if op == OP_IHS and (n_haps is None or len(n_haps) != len(outs)):
        raise ValueError("iHS scans need their haplotype counts")
    arr = (_StdRegion * len(outs))()
    dev = outs[0]["unstd"].device
    for i, o in enumerate(outs):
        M = int(o["unstd"].numel())
        for k, dt in (("unstd", torch.float64), ("status", torch.int8), ("std", torch.float64)):
            if o[k].dtype != dt or o[k].numel() != M or not o[k].is_contiguous():
                raise ValueError("scan %d: %s must be a contiguous %s tensor of %d" % (i, k, dt, M))
        fr = o.get("freq") if op == OP_IHS else None
        if op == OP_IHS and (fr is None or fr.dtype != torch.float64 or fr.numel() != M):
            raise ValueError("scan %d: iHS scans need their float64 freq" % i)
        arr[i] = _StdRegion(o["unstd"].data_ptr(), fr.data_ptr() if fr is not None else None,
                            o["status"].data_ptr(), o["std"].data_ptr(), M,
                            int(n_haps[i]) if op == OP_IHS else 0, 0)
    cp = _cparams(params)
    nb = lib().ss_genome_workspace_bytes(arr, len(outs), op, ctypes.byref(cp))
    if nb == 0:
        raise SelscanError(SS_EARG, "invalid arguments for ss_genome_workspace_bytes: " +
                           lib().ss_last_error().decode())
    ws = _workspace(nb, dev, ws)
    base = _aligned(ws)
    nbins = int(math.floor(1.0 / (params or Params()).bin_width + 0.5)) if op == OP_IHS else 1
    binstat = torch.empty((max(1, nbins), 3), dtype=torch.float64, device=dev)
    _check(lib().ss_genome_standardize(arr, len(outs), op, ctypes.byref(cp), _ptr(binstat),
                                       ctypes.c_void_p(base), ws.numel() - (base - ws.data_ptr()),
                                       _stream(stream)))
    return binstat


# ---- measurement kernels (include/selscan_micro.h) ------------------------------

def micro(rows: torch.Tensor, copy_bytes: int = 1 << 30, stream=None) -> dict:
    """Achievable rates of the GPU resources the walks use, measured on the
    current device: HBM stream copy (GB/s), int32 VALU (T lane-ops/s), LDS
    atomics (G ops/s) and the cell-update proxy (G cells/s) over ``rows``
    (device uint64 [n_rows, 4], e.g. a packed 204-haplotype matrix)."""
    L = lib()
    dev = rows.device
    if rows.dtype != torch.int64 or rows.dim() != 2 or rows.shape[1] != 4 or not rows.is_contiguous():
        raise ValueError("rows must be a contiguous int64 tensor [n_rows, 4]")
    out = torch.zeros(L.ss_micro_out_words(), dtype=torch.int32, device=dev)
    ms, x = ctypes.c_double(0.0), ctypes.c_double(0.0)
    src = torch.empty(copy_bytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(copy_bytes, dtype=torch.uint8, device=dev)
    st = _stream(stream)
    _check(L.ss_micro_copy(_ptr(src), _ptr(dst), copy_bytes, 10, st, ctypes.byref(ms)))
    res = {"hbm_copy_GBps": round(2.0 * copy_bytes / (ms.value * 1e-3) / 1e9, 1),
           "hbm_copy_bytes": copy_bytes}
    del src, dst
    _check(L.ss_micro_valu(_ptr(out), 4096, 10, st, ctypes.byref(ms), ctypes.byref(x)))
    res["valu_int32_TOPs"] = round(x.value / (ms.value * 1e-3) / 1e12, 3)
    _check(L.ss_micro_lds_atomic(_ptr(out), 4096, 10, st, ctypes.byref(ms), ctypes.byref(x)))
    res["lds_atomic_Gops"] = round(x.value / (ms.value * 1e-3) / 1e9, 1)
    _check(L.ss_micro_cell(_ptr(rows), rows.shape[0], _ptr(out), 2048, 10, st, ctypes.byref(ms),
                           ctypes.byref(x)))
    res["cell_proxy_Gcells"] = round(x.value / (ms.value * 1e-3) / 1e9, 1)
    return res


def static_scratch_bytes() -> int:
    return int(lib().ss_static_scratch_bytes())


def xpehh(a: HapMat, b: HapMat, params: Optional[Params] = None, steps: bool = False,
          stream=None, ws: Optional[torch.Tensor] = None, out: Optional[dict] = None,
          validate: bool = True):
    """XPEHH scan of population a against b (Sec. 1.3).  Returns ihhA, ihhB,
    unstd, std (float64), status (int8) and optionally steps (int32 [M, 2])."""
    if validate:
        a.validate()
        b.validate()
        if a.n_sites != b.n_sites or not torch.equal(a.pos_bp, b.pos_bp) \
                or not torch.equal(a.gpos_cm, b.gpos_cm):
            raise ValueError("XPEHH populations must share their sites")
    da, db = a.desc(), b.desc()
    M = a.n_sites
    dev = a.bits.device
    nb = workspace_bytes(OP_XPEHH, a, b, params)
    ws = _workspace(nb, dev, ws)
    if out is None:
        out = {k: torch.empty(M, dtype=torch.float64, device=dev)
               for k in ("ihhA", "ihhB", "unstd", "std")}
        out["status"] = torch.empty(M, dtype=torch.int8, device=dev)
        if steps:
            out["steps"] = torch.empty((M, 2), dtype=torch.int32, device=dev)
    cp = _cparams(params)
    base = _aligned(ws)
    avail = ws.numel() - (base - ws.data_ptr())
    _check(lib().ss_xpehh(ctypes.byref(da), ctypes.byref(db), ctypes.byref(cp),
                          _ptr(out["ihhA"]), _ptr(out["ihhB"]), _ptr(out["unstd"]),
                          _ptr(out["std"]), _ptr(out["status"]), _ptr(out.get("steps")),
                          ctypes.c_void_p(base), avail, _stream(stream)))
    return out


def ehh(h: HapMat, core: int, params: Optional[Params] = None, cap: int = 4096,
        sizes: bool = False, stream=None):
    """EHH curves at one core site (Sec. 1.1), both directions.  Returns S
    (uint64 as int64 [2, cap+1, 2]), ehh (float64 [2, cap+1, 3]), len
    (int64 [2]), optionally sizes (int32 view of uint32 [2, cap+1, n]),
    ihh (float64 [2] = iHH_0, iHH_1) and status (int8 [1])."""
    d = h.desc()
    dev = h.bits.device
    nb = workspace_bytes(OP_EHH, h, None, params, cap)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    out = {
        "S": torch.empty((2, cap + 1, 2), dtype=torch.int64, device=dev),
        "ehh": torch.empty((2, cap + 1, 3), dtype=torch.float64, device=dev),
        "len": torch.empty(2, dtype=torch.int64, device=dev),
        "ihh": torch.empty(2, dtype=torch.float64, device=dev),
        "status": torch.empty(1, dtype=torch.int8, device=dev),
    }
    if sizes:
        out["sizes"] = torch.empty((2, cap + 1, h.n_haps), dtype=torch.int32, device=dev)
    cp = _cparams(params)
    base = _aligned(ws)
    _check(lib().ss_ehh(ctypes.byref(d), int(core), ctypes.byref(cp), int(cap), _ptr(out["S"]),
                        _ptr(out["ehh"]), _ptr(out["len"]), _ptr(out.get("sizes")),
                        _ptr(out["ihh"]), _ptr(out["status"]), ctypes.c_void_p(base),
                        ws.numel() - (base - ws.data_ptr()), _stream(stream)))
    return out


WALK_AUTO, WALK_LDS_IDS, WALK_REG_MASKS, WALK_WIDE = 0, 1, 2, 3


def set_walk_kernel(kind: int):
    """Select the EHH-walk kernel (0 auto, 1 class ids in LDS, 2 register
    bitmasks, 3 the persistent list walk)."""
    _check(lib().ss_set_walk_kernel(int(kind)))


# ---- batched scans ------------------------------------------------------------------

@dataclasses.dataclass
class ScanRequest:
    """One region of a batch: iHS over ``a`` (b None) or XPEHH of a against b.
    ``out`` holds the device outputs (allocated by :func:`alloc_outputs`)."""
    a: HapMat
    b: Optional[HapMat] = None
    out: Optional[dict] = None

    @property
    def op(self) -> int:
        return OP_IHS if self.b is None else OP_XPEHH


def alloc_outputs(req: ScanRequest, steps: bool = False) -> dict:
    M = req.a.n_sites
    dev = req.a.bits.device
    if req.b is None:
        names = ("ihh1", "ihh0", "unstd", "std", "freq")
    else:
        names = ("ihhA", "ihhB", "unstd", "std")
    out = {k: torch.empty(M, dtype=torch.float64, device=dev) for k in names}
    out["status"] = torch.empty(M, dtype=torch.int8, device=dev)
    if steps:
        shape = (M, 2, 2) if req.b is None else (M, 2)
        out["steps"] = torch.empty(shape, dtype=torch.int32, device=dev)
    req.out = out
    return out


def _requests(reqs):
    arr = (_Request * len(reqs))()
    empty = _HapMat(None, 0, 0, 0, None, None)
    for i, r in enumerate(reqs):
        o = r.out
        if o is None:
            raise ValueError("request %d has no outputs (alloc_outputs)" % i)
        if r.b is None:
            x, y, f = o["ihh1"], o["ihh0"], o["freq"]
        else:
            x, y, f = o["ihhA"], o["ihhB"], None
        arr[i] = _Request(r.op, r.a.desc(), r.b.desc() if r.b is not None else empty,
                          x.data_ptr(), y.data_ptr(), o["unstd"].data_ptr(), o["std"].data_ptr(),
                          f.data_ptr() if f is not None else None, o["status"].data_ptr(),
                          o["steps"].data_ptr() if "steps" in o else None)
    return arr


def batch_workspace_bytes(reqs, params: Optional[Params] = None) -> int:
    arr = _requests(reqs)
    cp = _cparams(params)
    n = lib().ss_batch_workspace_bytes(arr, len(reqs), ctypes.byref(cp))
    if n == 0:
        raise SelscanError(SS_EARG, lib().ss_last_error().decode() or "invalid batch")
    return int(n)


def scan_batch(reqs, params: Optional[Params] = None, stream=None,
               ws: Optional[torch.Tensor] = None, validate: bool = True):
    """Scan every request of ``reqs`` (a list of ScanRequest with outputs)
    in one sequence; the EHH walks of all regions run in one persistent
    launch.  Returns the workspace tensor (reuse it for the next call)."""
    if validate:
        for r in reqs:
            r.a.validate()
            if r.b is not None:
                r.b.validate()
                if r.a.n_sites != r.b.n_sites or not torch.equal(r.a.pos_bp, r.b.pos_bp) \
                        or not torch.equal(r.a.gpos_cm, r.b.gpos_cm):
                    raise ValueError("XPEHH populations must share their sites")
    arr = _requests(reqs)
    cp = _cparams(params)
    nb = lib().ss_batch_workspace_bytes(arr, len(reqs), ctypes.byref(cp))
    if nb == 0:
        raise SelscanError(SS_EARG, lib().ss_last_error().decode() or "invalid batch")
    dev = reqs[0].a.bits.device
    ws = _workspace(int(nb), dev, ws)
    base = _aligned(ws)
    _check(lib().ss_scan_batch(arr, len(reqs), ctypes.byref(cp), ctypes.c_void_p(base),
                               ws.numel() - (base - ws.data_ptr()), _stream(stream)))
    return ws


@dataclasses.dataclass
class BatchConfig:
    """Launch configuration of the persistent walk (see ss_batch_config)."""
    threads: int = 64
    pair_cap: int = 4096
    chunk: int = 1
    blocks_per_cu: int = 0
    order: int = 0
    small_kernel: int = 1
    kernel: int = 0
    small_pair_cap: int = 1024
    slots: int = 16
    class_cap: int = 256
    counter_copies: int = 0


def get_batch_config() -> BatchConfig:
    c = _BatchConfig()
    _check(lib().ss_get_batch_config(ctypes.byref(c)))
    return BatchConfig(c.threads, c.pair_cap, c.chunk, c.blocks_per_cu, c.order, c.small_kernel,
                       c.kernel, c.small_pair_cap, c.slots, c.class_cap, c.counter_copies)


def set_batch_config(cfg: BatchConfig):
    c = _BatchConfig(int(cfg.threads), int(cfg.pair_cap), int(cfg.chunk), int(cfg.blocks_per_cu),
                     int(cfg.order), int(cfg.small_kernel), int(cfg.kernel),
                     int(cfg.small_pair_cap), int(cfg.slots), int(cfg.class_cap),
                     int(cfg.counter_copies))
    _check(lib().ss_set_batch_config(ctypes.byref(c)))


def group_tuning() -> list:
    """Settings the autotuner refined per launch group: a list of dicts
    {threads, pairs, counter_copies, class_cap, chunk, blocks_per_cu, plain}."""
    n = ctypes.c_int32(0)
    _check(lib().ss_get_group_tuning(None, 0, ctypes.byref(n)))
    rows = (ctypes.c_int32 * (7 * max(1, n.value)))()
    _check(lib().ss_get_group_tuning(rows, n.value, ctypes.byref(n)))
    return [dict(zip(_TUNE_KEYS, rows[7 * i: 7 * i + 7])) for i in range(n.value)]


_TUNE_KEYS = ("threads", "pairs", "counter_copies", "class_cap", "chunk", "blocks_per_cu", "plain")


def set_group_tuning(rows: list):
    """Replace the per-launch-group settings (dicts with the keys group_tuning
    returns; an empty list drops them)."""
    flat = [int(r[k]) for r in rows for k in _TUNE_KEYS]
    arr = (ctypes.c_int32 * max(1, len(flat)))(*flat)
    _check(lib().ss_set_group_tuning(arr, len(rows)))


def autotune_batch(reqs, params: Optional[Params] = None, stream=None,
                   ws: Optional[torch.Tensor] = None, sample_items: int = 0):
    """Time configurations of the persistent walk on these requests and keep
    the fastest (process-wide).  Returns (BatchConfig, ms, workspace)."""
    arr = _requests(reqs)
    cp = _cparams(params)
    nb = lib().ss_batch_workspace_bytes(arr, len(reqs), ctypes.byref(cp))
    if nb == 0:
        raise SelscanError(SS_EARG, lib().ss_last_error().decode() or "invalid batch")
    ws = _workspace(int(nb), reqs[0].a.bits.device, ws)
    base = _aligned(ws)
    best = _BatchConfig()
    ms = ctypes.c_double(0.0)
    _check(lib().ss_autotune_batch(arr, len(reqs), ctypes.byref(cp), ctypes.c_void_p(base),
                                   ws.numel() - (base - ws.data_ptr()), _stream(stream),
                                   int(sample_items), ctypes.byref(best), ctypes.byref(ms)))
    cfg = BatchConfig(best.threads, best.pair_cap, best.chunk, best.blocks_per_cu, best.order,
                      best.small_kernel, best.kernel, best.small_pair_cap, best.slots,
                      best.class_cap, best.counter_copies)
    return cfg, float(ms.value), ws


def set_graph(on: bool = True):
    """Capture scan_batch sequences into HIP graphs and replay them."""
    _check(lib().ss_set_graph(1 if on else 0))


def graph_clear():
    _check(lib().ss_graph_clear())


def set_mask_lanes(lanes_per_class: int):
    """Lanes per class of the bitmask walk (1, 2, 4, 8; 0 = default)."""
    _check(lib().ss_set_mask_lanes(int(lanes_per_class)))


def set_mask_skip(max_classes: int):
    """Bitmask walk: batches with at most ``max_classes`` live classes refine
    only the markers that cut a class (0 .. 64; 0 refines every marker)."""
    _check(lib().ss_set_mask_skip(int(max_classes)))


def timing_enable(on: bool = True):
    _check(lib().ss_timing_enable(1 if on else 0))


def timing_read(reset: bool = False):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().ss_timing_read(ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return float(ms.value), int(n.value)


def version() -> str:
    return lib().ss_version().decode()
