"""ctypes binding of libbandops.so (include/bandops.h).

Argument marshalling only: every operator runs in the library's HIP kernels on
the caller's current torch stream; torch provides device memory.  Band arrays
are torch tensors of shape (n, ld) -- row j is record j, column j of the matrix
restricted to its band (slot u+i-j holds element (i,j)).  In the mixed format a
band is a float32 tensor plus an FP64 diagonal tensor of length n.

Importing this module does not touch the GPU; the first call loads the library
and raises RuntimeError if it is missing (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BANDOPS_LIB") or os.path.join(_HERE, "libbandops.so")

F64, MIXED = 0, 1
KMAX = 12
SCALE_BAND, SCALE_BAND_SYM, SCALE_VEC, SCALE_PROBLEM = 0, 1, 2, 3

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


class _Band(ctypes.Structure):
    _fields_ = [("band", _P), ("diag64", _P), ("n", _I64), ("l", _I32), ("u", _I32),
                ("ld", _I32), ("reserved", _I32)]


class _Problem(ctypes.Structure):
    _fields_ = [("n", _I64), ("k", _I32), ("reserved", _I32), ("boff", _I64), ("voff", _I64)]


class _BatchIO(ctypes.Structure):
    _fields_ = [(name, _P) for name in (
        "Q", "Qd", "y", "S", "Sd", "L", "Ld", "z", "x", "Sig", "Sigd", "Lbar", "Lbard",
        "Qbar", "Qbard", "logdet", "parts", "info", "loss", "Sbar", "Sbard")]


class _MLIO(ctypes.Structure):
    _fields_ = [(name, _P) for name in (
        "Q", "Qd", "mask", "b", "tau2", "L", "Ld", "Sig", "Sigd", "x", "Qbar", "Qbard", "bbar", "tau2bar",
        "parts", "info")]


class _NGIO(ctypes.Structure):
    _fields_ = [(name, _P) for name in (
        "Lpr", "Lprd", "etapr", "Llik", "Llikd", "etalik", "L", "Ld", "Sig", "Sigd", "x", "Lprbar", "Lprbard",
        "Llikbar", "Llikbard", "etaprbar", "parts", "info")]


class _WHIO(ctypes.Structure):
    _fields_ = [(name, _P) for name in (
        "Q", "Qd", "v", "L", "Ld", "F", "Fbar", "vbar", "Qbar", "Qbard", "logdet", "info")] + [("reuse", _I32)]


class _KLIO(ctypes.Structure):
    _fields_ = [(name, _P) for name in (
        "Lq", "Lqd", "Lp", "Lpd", "mq", "mp", "Sig", "Sigd", "Lqbar", "Lqbard", "Lpbar", "Lpbard",
        "mqbar", "mpbar", "parts")]


_lib = None


def lib():
    """Load libbandops.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libbandops.so not found at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    bp = ctypes.POINTER(_Band)
    sigs = {
        "bo_workspace_size": (ctypes.c_size_t, [_I64, _I32]),
        "bo_chol": (_I32, [_I32, bp, bp, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
        "bo_chol_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "bo_chol_noalloc": (_I32, [_I32, bp, bp, _P, _P, _P, _P, _P]),
        "bo_trsv": (_I32, [_I32, bp, _I32, _P, _P, _I64, _I64, _P, ctypes.c_size_t, _P]),
        "bo_subset_inv_workspace_size": (ctypes.c_size_t, [_I64, _I32, _I32]),
        "bo_subset_inv": (_I32, [_I32, bp, bp, _P, ctypes.c_size_t, _P]),
        "bo_gbmm": (_I32, [_I32, bp, _I32, bp, _I32, bp, _P]),
        "bo_gbmv": (_I32, [_I32, bp, _I32, _P, _P, _P]),
        "bo_outer_band": (_I32, [_I32, _P, _P, ctypes.c_double, _I32, bp, _P]),
        "bo_solve_band_mat": (_I32, [_I32, bp, bp, bp, _P]),
        "bo_solve_band_mat_workspace": (ctypes.c_size_t, [_I64, _I32, _I32]),
        "bo_solve_band_mat_bwd": (_I32, [_I32, bp, bp, bp, bp, bp, _P, ctypes.c_size_t, _P]),
        "bo_chol_bwd": (_I32, [_I32, bp, bp, bp, _P, ctypes.c_size_t, _P]),
        "bo_subset_inv_bwd": (_I32, [_I32, bp, bp, bp, bp, _I32, _P, ctypes.c_size_t, _P]),
        "bo_trsv_bwd": (_I32, [_I32, bp, _I32, _P, _P, _P, bp, _I32, _P, ctypes.c_size_t, _P]),
        "bo_logdet_bwd": (_I32, [_I32, bp, _P, bp, _I32, _P]),
        "bo_plan_create": (_I32, [ctypes.POINTER(_Problem), _I32, _I64, ctypes.POINTER(_P)]),
        "bo_plan_workspace_size": (_I32, [_P, ctypes.POINTER(ctypes.c_size_t)]),
        "bo_plan_loss_workspace_size": (_I32, [_P, ctypes.POINTER(ctypes.c_size_t)]),
        "bo_plan_upload": (_I32, [_P, _P, _P]),
        "bo_plan_forward": (_I32, [_P, _I32, ctypes.POINTER(_BatchIO), _P, _P]),
        "bo_plan_gauss_loss": (_I32, [_P, _I32, ctypes.POINTER(_BatchIO), _P, _P]),
        "bo_plan_vi_kl": (_I32, [_P, _I32, ctypes.POINTER(_KLIO), _P, _P]),
        "bo_plan_marglik": (_I32, [_P, _I32, ctypes.POINTER(_MLIO), _P, _P]),
        "bo_plan_natgp": (_I32, [_P, _I32, ctypes.POINTER(_NGIO), _P, _P]),
        "bo_plan_whiten": (_I32, [_P, _I32, ctypes.POINTER(_WHIO), _P, _P]),
        "bo_rcm": (_I32, [_I64, _P, _P, _P, _P, _P]),
        "bo_csr_permute": (_I32, [_I64, _P, _P, _P, _P, _P, _P, _P]),
        "bo_csr_to_band": (_I32, [_I32, _I64, _I32, _P, _P, _I64, _P, _I32, _I64, _P, _P, _P, _P]),
        "bo_band_to_csr_grad": (_I32, [_I32, _I64, _I32, _P, _P, _I64, _I32, _I64, _P, _P, _P, _P]),
        "bo_plan_whiten_bwd": (_I32, [_P, _I32, ctypes.POINTER(_WHIO), _P, _P]),
        "bo_plan_scale": (_I32, [_P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
        "bo_plan_stats": (_I32, [_P, ctypes.POINTER(_I64)]),
        "bo_plan_destroy": (_I32, [_P]),
        "bo_wide_workspace_size": (_I32, [ctypes.POINTER(_Problem), _I32, ctypes.POINTER(ctypes.c_size_t)]),
        "bo_wide_upload": (_I32, [ctypes.POINTER(_Problem), _I32, _P, ctypes.c_size_t]),
        "bo_wide_forward": (_I32, [ctypes.POINTER(_Problem), _I32, ctypes.POINTER(_BatchIO), _P, ctypes.c_size_t,
                                    _P]),
        "bo_wide_gauss_loss": (_I32, [ctypes.POINTER(_Problem), _I32, ctypes.POINTER(_BatchIO), _P,
                                       ctypes.c_size_t, _P]),
        "bo_profile_enable": (_I32, [_I32]),
        "bo_profile_read": (_I32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64), _I32]),
        "bo_profile_slots": (_I32, []),
        "bo_profile_slot_name": (ctypes.c_char_p, [_I32]),
        "bo_status_string": (ctypes.c_char_p, [_I32]),
        "bo_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ("bo_workspace_size", "bo_chol", "bo_chol_noalloc_scratch_bytes", "bo_chol_noalloc", "bo_trsv", "bo_subset_inv_workspace_size", "bo_subset_inv", "bo_gbmm", "bo_gbmv",
            "bo_outer_band", "bo_solve_band_mat", "bo_solve_band_mat_workspace",
            "bo_solve_band_mat_bwd", "bo_chol_bwd", "bo_subset_inv_bwd", "bo_trsv_bwd", "bo_logdet_bwd",
            "bo_plan_create", "bo_plan_workspace_size", "bo_plan_loss_workspace_size", "bo_plan_upload", "bo_plan_forward",
            "bo_plan_gauss_loss", "bo_plan_vi_kl", "bo_plan_marglik", "bo_plan_natgp", "bo_plan_whiten", "bo_plan_whiten_bwd", "bo_rcm", "bo_csr_permute", "bo_csr_to_band", "bo_band_to_csr_grad", "bo_plan_scale", "bo_plan_stats", "bo_plan_destroy", "bo_wide_workspace_size",
            "bo_wide_upload", "bo_wide_forward", "bo_wide_gauss_loss", "bo_profile_enable",
            "bo_profile_read", "bo_profile_slots", "bo_profile_slot_name", "bo_status_string",
            "bo_last_error")


class BandOpsError(RuntimeError):
    pass


def _check(status: int, what: str):
    if status != 0:
        L = lib()
        raise BandOpsError(f"{what}: {L.bo_status_string(status).decode()} "
                           f"({L.bo_last_error().decode()})")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Band:
    """A band on the device: `band` (n, ld) float64 (F64) or float32 (mixed,
    then `diag` holds the FP64 diagonal), lower width l, upper width u."""
    band: torch.Tensor
    l: int
    u: int = 0
    diag: Optional[torch.Tensor] = None

    @property
    def n(self):
        return self.band.shape[0]

    @property
    def prec(self):
        return MIXED if self.band.dtype == torch.float32 else F64

    def c(self) -> _Band:
        b = self.band
        if not b.is_contiguous():
            raise ValueError("band tensors must be contiguous")
        return _Band(_ptr(b), _ptr(self.diag), b.shape[0], self.l, self.u, b.shape[1], 0)

    def dense_slots(self) -> torch.Tensor:
        """FP64 view of the records with the FP64 diagonal in its slot."""
        out = self.band.double().clone()
        if self.diag is not None:
            out[:, self.u] = self.diag
        return out


def new_band(n: int, l: int, u: int = 0, prec: int = F64, device="cuda") -> Band:
    if prec == F64:
        return Band(torch.zeros((n, l + u + 1), dtype=torch.float64, device=device), l, u)
    return Band(torch.zeros((n, l + u + 1), dtype=torch.float32, device=device), l, u,
                torch.zeros(n, dtype=torch.float64, device=device))


def band_from(t: torch.Tensor, l: int, u: int = 0, prec: int = F64) -> Band:
    """Band from an FP64 (n, l+u+1) tensor; mixed keeps the diagonal in FP64."""
    if prec == F64:
        return Band(t.to(torch.float64).contiguous(), l, u)
    return Band(t.to(torch.float32).contiguous(), l, u, t[:, u].to(torch.float64).contiguous())


def _vec_dtype(prec):
    return torch.float64 if prec == F64 else torch.float32


_ws_cache = {}


def workspace(n: int, k: int) -> torch.Tensor:
    """Device workspace for a single-problem call (cached per device and size;
    calls are ordered on the current stream, so reuse is safe there)."""
    size = max(int(lib().bo_workspace_size(n, k)), 256)
    dev = torch.device("cuda", torch.cuda.current_device())
    key = (dev.index, size)
    t = _ws_cache.get(key)
    if t is None:
        _ws_cache.clear()
        t = torch.empty(size, dtype=torch.uint8, device=dev)
        _ws_cache[key] = t
    return t


# ------------------------------------------------------------ forward ops

def bo_chol(Q: Band, y: Optional[torch.Tensor] = None):
    """C + log det (+ z = L^{-1} y).  Returns (L, z, logdet, info) (device)."""
    prec = Q.prec
    L = new_band(Q.n, Q.l, 0, prec, Q.band.device)
    z = torch.empty_like(y) if y is not None else None
    logdet = torch.zeros(1, dtype=torch.float64, device=Q.band.device)
    info = torch.zeros(1, dtype=torch.int32, device=Q.band.device)
    ws = workspace(Q.n, Q.l)
    qc, lc = Q.c(), L.c()
    _check(lib().bo_chol(prec, ctypes.byref(qc), ctypes.byref(lc), _ptr(y), _ptr(z), _ptr(logdet),
                         _ptr(info), _ptr(ws), ws.numel(), _stream()), "bo_chol")
    return L, z, logdet, info


def bo_chol_noalloc(Q: Band, y: Optional[torch.Tensor] = None, out=None):
    """bo_chol with the library's fixed scratch array as its workspace (no
    workspace argument, no allocation inside the call).  out: optional (L, z,
    logdet, info) tensors to write into (the caller allocates them once);
    returns them."""
    prec = Q.prec
    if out is None:
        L = new_band(Q.n, Q.l, 0, prec, Q.band.device)
        z = torch.empty_like(y) if y is not None else None
        logdet = torch.zeros(1, dtype=torch.float64, device=Q.band.device)
        info = torch.zeros(1, dtype=torch.int32, device=Q.band.device)
    else:
        L, z, logdet, info = out
    qc, lc = Q.c(), L.c()
    _check(lib().bo_chol_noalloc(prec, ctypes.byref(qc), ctypes.byref(lc), _ptr(y), _ptr(z), _ptr(logdet),
                                 _ptr(info), _stream()), "bo_chol_noalloc")
    return L, z, logdet, info


def bo_trsv(L: Band, b: torch.Tensor, trans: int = 0):
    """X = L^{-1} B or L^{-T} B; b is one vector (n,) or nrhs columns stored
    as rows of a (nrhs, n) tensor (column c at element c * n)."""
    b = b.contiguous()
    x = torch.empty_like(b)
    nrhs, ldx = (1, L.n) if b.dim() == 1 else (b.shape[0], b.shape[1])
    ws = workspace(L.n, L.l)
    lc = L.c()
    _check(lib().bo_trsv(L.prec, ctypes.byref(lc), int(trans), _ptr(b), _ptr(x), int(nrhs), int(ldx), _ptr(ws),
                         ws.numel(), _stream()), "bo_trsv")
    return x


def bo_subset_inv(L: Band, kout: Optional[int] = None):
    """Lower band of (L L^T)^{-1} of width kout (default: L's own width)."""
    kout = L.l if kout is None else int(kout)
    S = new_band(L.n, kout, 0, L.prec, L.band.device)
    if kout == L.l:
        ws = workspace(L.n, L.l)
    else:
        size = max(int(lib().bo_subset_inv_workspace_size(L.n, L.l, kout)), 256)
        ws = torch.empty(size, dtype=torch.uint8, device=L.band.device)
    lc, sc = L.c(), S.c()
    _check(lib().bo_subset_inv(L.prec, ctypes.byref(lc), ctypes.byref(sc), _ptr(ws), ws.numel(),
                               _stream()), "bo_subset_inv")
    return S


def bo_gbmm(A: Band, B: Band, tA: int = 0, tB: int = 0, l: Optional[int] = None,
            u: Optional[int] = None):
    lA, uA = (A.u, A.l) if tA else (A.l, A.u)
    lB, uB = (B.u, B.l) if tB else (B.l, B.u)
    l = lA + lB if l is None else l
    u = uA + uB if u is None else u
    C = new_band(A.n, l, u, A.prec, A.band.device)
    ac, bc, cc = A.c(), B.c(), C.c()
    _check(lib().bo_gbmm(A.prec, ctypes.byref(ac), int(tA), ctypes.byref(bc), int(tB),
                         ctypes.byref(cc), _stream()), "bo_gbmm")
    return C


def bo_gbmv(A: Band, x: torch.Tensor, tA: int = 0):
    y = torch.empty_like(x)
    ac = A.c()
    _check(lib().bo_gbmv(A.prec, ctypes.byref(ac), int(tA), _ptr(x), _ptr(y), _stream()), "bo_gbmv")
    return y


def bo_outer_band(m: torch.Tensor, v: torch.Tensor, l: int, u: int = 0, alpha: float = 1.0,
                  out: Optional[Band] = None, accumulate: bool = False):
    prec = F64 if m.dtype == torch.float64 else MIXED
    O = out if out is not None else new_band(m.shape[0], l, u, prec, m.device)
    oc = O.c()
    _check(lib().bo_outer_band(prec, _ptr(m), _ptr(v), float(alpha), int(accumulate),
                               ctypes.byref(oc), _stream()), "bo_outer_band")
    return O


def bo_solve_band_mat(L: Band, R: Band):
    """Algorithm 5: the band (L.l lower, R.u upper) of L^{-1} R."""
    O = new_band(L.n, L.l, R.u, L.prec, L.band.device)
    lc, rc, oc = L.c(), R.c(), O.c()
    _check(lib().bo_solve_band_mat(L.prec, ctypes.byref(lc), ctypes.byref(rc), ctypes.byref(oc), _stream()),
           "bo_solve_band_mat")
    return O


# ----------------------------------------------------------- reverse mode

def bo_solve_band_mat_bwd(L: Band, O: Band, Obar: Band, lr: int):
    """Reverse mode of Algorithm 5 (Table 1, solve matrix-matrix): (Rbar on
    the band (lr, O.u), Lbar)."""
    Rbar = new_band(L.n, lr, O.u, L.prec, L.band.device)
    Lbar = new_band(L.n, L.l, 0, L.prec, L.band.device)
    size = max(int(lib().bo_solve_band_mat_workspace(L.n, L.l, O.u)), 256)
    ws = torch.empty(size, dtype=torch.uint8, device=L.band.device)
    lc, oc, obc, rbc, lbc = L.c(), O.c(), Obar.c(), Rbar.c(), Lbar.c()
    _check(lib().bo_solve_band_mat_bwd(L.prec, ctypes.byref(lc), ctypes.byref(oc), ctypes.byref(obc),
                                       ctypes.byref(rbc), ctypes.byref(lbc), _ptr(ws), ws.numel(), _stream()),
           "bo_solve_band_mat_bwd")
    return Rbar, Lbar


def bo_chol_bwd(L: Band, Lbar: Band):
    Qbar = new_band(L.n, L.l, 0, L.prec, L.band.device)
    ws = workspace(L.n, L.l)
    lc, lbc, qc = L.c(), Lbar.c(), Qbar.c()
    _check(lib().bo_chol_bwd(L.prec, ctypes.byref(lc), ctypes.byref(lbc), ctypes.byref(qc), _ptr(ws),
                             ws.numel(), _stream()), "bo_chol_bwd")
    return Qbar


def bo_subset_inv_bwd(L: Band, S: Band, Sbar: Band, out: Optional[Band] = None,
                      accumulate: bool = False):
    Lbar = out if out is not None else new_band(L.n, L.l, 0, L.prec, L.band.device)
    ws = workspace(L.n, L.l)
    lc, sc, sbc, lbc = L.c(), S.c(), Sbar.c(), Lbar.c()
    _check(lib().bo_subset_inv_bwd(L.prec, ctypes.byref(lc), ctypes.byref(sc), ctypes.byref(sbc),
                                   ctypes.byref(lbc), int(accumulate), _ptr(ws), ws.numel(),
                                   _stream()), "bo_subset_inv_bwd")
    return Lbar


def bo_trsv_bwd(L: Band, x: torch.Tensor, xbar: torch.Tensor, trans: int = 0,
                out: Optional[Band] = None, accumulate: bool = False):
    bbar = torch.empty_like(xbar)
    Lbar = out if out is not None else new_band(L.n, L.l, 0, L.prec, L.band.device)
    ws = workspace(L.n, L.l)
    lc, lbc = L.c(), Lbar.c()
    _check(lib().bo_trsv_bwd(L.prec, ctypes.byref(lc), int(trans), _ptr(x), _ptr(xbar), _ptr(bbar),
                             ctypes.byref(lbc), int(accumulate), _ptr(ws), ws.numel(), _stream()),
           "bo_trsv_bwd")
    return bbar, Lbar


def bo_logdet_bwd(L: Band, gbar: torch.Tensor, out: Optional[Band] = None, accumulate: bool = False):
    Lbar = out if out is not None else new_band(L.n, L.l, 0, L.prec, L.band.device)
    lc, lbc = L.c(), Lbar.c()
    g = gbar.reshape(1).to(torch.float64).contiguous()
    _check(lib().bo_logdet_bwd(L.prec, ctypes.byref(lc), _ptr(g), ctypes.byref(lbc), int(accumulate),
                               _stream()), "bo_logdet_bwd")
    return Lbar


# -------------------------------------------------------------- profiling

def profile_enable(on: bool = True):
    _check(lib().bo_profile_enable(int(on)), "bo_profile_enable")


def profile_read():
    """{step name: (total ms, launches)} since the last read (waits for the GPU)."""
    L = lib()
    n = L.bo_profile_slots()
    ms = (ctypes.c_double * n)()
    cnt = (_I64 * n)()
    _check(L.bo_profile_read(ms, cnt, n), "bo_profile_read")
    return {L.bo_profile_slot_name(i).decode(): (ms[i], cnt[i]) for i in range(n) if cnt[i]}


# ------------------------------------------------------------------ plans

class Plan:
    """Batched uneven problems: packed band arrays (problem p's records, stride
    k_p + 1, follow problem p-1's) and packed vectors."""

    def __init__(self, ns, ks, target_chunks: int = 0, device="cuda"):
        self.ns = [int(v) for v in ns]
        self.ks = [int(v) for v in ks]
        self.nprob = len(self.ns)
        probs = (_Problem * self.nprob)()
        boff = voff = 0
        self.boff, self.voff = [], []
        for i, (n, k) in enumerate(zip(self.ns, self.ks)):
            probs[i] = _Problem(n, k, 0, boff, voff)
            self.boff.append(boff)
            self.voff.append(voff)
            boff += n * (k + 1)
            voff += n
        self.band_elems, self.rows = boff, voff
        h = _P()
        _check(lib().bo_plan_create(probs, self.nprob, int(target_chunks), ctypes.byref(h)),
               "bo_plan_create")
        self.h = h
        sz = ctypes.c_size_t()
        _check(lib().bo_plan_workspace_size(h, ctypes.byref(sz)), "bo_plan_workspace_size")
        self.ws = torch.empty(max(sz.value, 256), dtype=torch.uint8, device=device)
        _check(lib().bo_plan_upload(h, _ptr(self.ws), _stream()), "bo_plan_upload")
        st = (_I64 * 5)()
        _check(lib().bo_plan_stats(h, st), "bo_plan_stats")
        self.stats = dict(nprob=st[0], nchunk=st[1], ngroup=st[2], rows=st[3], kmax=st[4])

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and _lib is not None:
                _lib.bo_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def io(self, **arrays) -> _BatchIO:
        io = _BatchIO()
        for k_, v in arrays.items():
            setattr(io, k_, _ptr(v))
        return io

    def forward(self, prec: int, io: _BatchIO):
        _check(lib().bo_plan_forward(self.h, prec, ctypes.byref(io), _ptr(self.ws), _stream()),
               "bo_plan_forward")

    def ensure_loss_workspace(self):
        """Grow the workspace to what bo_plan_gauss_loss needs when it keeps L,
        Sig and Lbar in it (io without L, Sig and Lbar); call before graph
        capture."""
        sz = ctypes.c_size_t()
        _check(lib().bo_plan_loss_workspace_size(self.h, ctypes.byref(sz)), "bo_plan_loss_workspace_size")
        if self.ws.numel() < sz.value:
            self.ws = torch.empty(sz.value, dtype=torch.uint8, device=self.ws.device)
            _check(lib().bo_plan_upload(self.h, _ptr(self.ws), _stream()), "bo_plan_upload")

    def gauss_loss(self, prec: int, io: _BatchIO):
        """The loss unit over the batch (bo_plan_gauss_loss).  An io without L,
        Sig and Lbar keeps them in the workspace (grown on first use)."""
        if not io.L and not io.Sig and not io.Lbar:
            self.ensure_loss_workspace()
        _check(lib().bo_plan_gauss_loss(self.h, prec, ctypes.byref(io), _ptr(self.ws), _stream()),
               "bo_plan_gauss_loss")

    def scale(self, prec: int, kind: int, g: Optional[torch.Tensor], inp: torch.Tensor,
              out: torch.Tensor, ind: Optional[torch.Tensor] = None, outd: Optional[torch.Tensor] = None):
        """out = g[p] * inp over every problem p (bo_plan_scale): kind
        SCALE_BAND / SCALE_BAND_SYM on packed records, SCALE_VEC on packed
        vectors, SCALE_PROBLEM on one FP64 value per problem; g None scales by
        1.  out may be inp."""
        _check(lib().bo_plan_scale(self.h, prec, int(kind), _ptr(g), _ptr(inp), _ptr(ind), _ptr(out), _ptr(outd),
                                   _ptr(self.ws), _stream()), "bo_plan_scale")
        return out

    def kl_io(self, **arrays) -> _KLIO:
        io = _KLIO()
        for k_, v in arrays.items():
            setattr(io, k_, _ptr(v))
        return io

    def vi_kl(self, prec: int, io: _KLIO):
        """KL term of the variational objective for every problem (see
        bo_plan_vi_kl): fills io.Sig, the four gradients and io.parts."""
        _check(lib().bo_plan_vi_kl(self.h, prec, ctypes.byref(io), _ptr(self.ws), _stream()),
               "bo_plan_vi_kl")

    def ml_io(self, **arrays) -> _MLIO:
        io = _MLIO()
        for k_, v in arrays.items():
            setattr(io, k_, _ptr(v))
        return io

    def marglik(self, prec: int, io: _MLIO):
        """Log marginal likelihood with partial observations and its reverse
        mode for every problem (see bo_plan_marglik): fills io.L, io.Sig, io.x,
        io.Qbar, io.bbar, io.tau2bar, io.parts and io.info."""
        _check(lib().bo_plan_marglik(self.h, prec, ctypes.byref(io), _ptr(self.ws), _stream()),
               "bo_plan_marglik")

    def ng_io(self, **arrays) -> _NGIO:
        io = _NGIO()
        for k_, v in arrays.items():
            setattr(io, k_, _ptr(v))
        return io

    def natgp(self, prec: int, io: _NGIO):
        """GP regression with banded natural parameters and its reverse mode
        for every problem (see bo_plan_natgp): fills io.L, io.Sig, io.x (the
        posterior mean, also the gradient in eta_lik), io.Lprbar, io.Llikbar,
        io.etaprbar, io.parts and io.info."""
        _check(lib().bo_plan_natgp(self.h, prec, ctypes.byref(io), _ptr(self.ws), _stream()), "bo_plan_natgp")

    def wh_io(self, reuse: bool = False, **arrays) -> _WHIO:
        """reuse: the backward call takes the chunk products of L that the
        preceding whiten call on this plan left in the workspace."""
        io = _WHIO()
        for k_, v in arrays.items():
            setattr(io, k_, _ptr(v))
        io.reuse = 1 if reuse else 0
        return io

    def whiten(self, prec: int, io: _WHIO):
        """Whitened sample F = L^{-T} v with L = C(Q) for every problem (see
        bo_plan_whiten): fills io.L, io.F and, when given, io.logdet, io.info."""
        _check(lib().bo_plan_whiten(self.h, prec, ctypes.byref(io), _ptr(self.ws), _stream()), "bo_plan_whiten")

    def whiten_bwd(self, prec: int, io: _WHIO):
        """Reverse mode of the whitened sample from io.Fbar (see
        bo_plan_whiten_bwd): fills io.vbar and io.Qbar."""
        _check(lib().bo_plan_whiten_bwd(self.h, prec, ctypes.byref(io), _ptr(self.ws), _stream()),
               "bo_plan_whiten_bwd")


class WidePlan:
    """Batched wide block-banded problems (k = 64, mixed storage): packed
    records of 65 FP32 values (problem p's follow problem p-1's), packed FP64
    diagonals and vectors."""

    K = 64

    def __init__(self, ns, device="cuda"):
        self.ns = [int(v) for v in ns]
        self.nprob = len(self.ns)
        probs = (_Problem * self.nprob)()
        boff = voff = 0
        self.boff, self.voff = [], []
        for i, n in enumerate(self.ns):
            probs[i] = _Problem(n, self.K, 0, boff, voff)
            self.boff.append(boff)
            self.voff.append(voff)
            boff += n * (self.K + 1)
            voff += n
        self.band_elems, self.rows = boff, voff
        self.probs = probs
        sz = ctypes.c_size_t()
        _check(lib().bo_wide_workspace_size(probs, self.nprob, ctypes.byref(sz)), "bo_wide_workspace_size")
        self.ws = torch.empty(max(sz.value, 256), dtype=torch.uint8, device=device)
        _check(lib().bo_wide_upload(probs, self.nprob, _ptr(self.ws), self.ws.numel()), "bo_wide_upload")

    def io(self, **arrays) -> _BatchIO:
        io = _BatchIO()
        for k_, v in arrays.items():
            setattr(io, k_, _ptr(v))
        return io

    def forward(self, io: _BatchIO):
        _check(lib().bo_wide_forward(self.probs, self.nprob, ctypes.byref(io), _ptr(self.ws), self.ws.numel(),
                                     _stream()), "bo_wide_forward")

    def gauss_loss(self, io: _BatchIO):
        _check(lib().bo_wide_gauss_loss(self.probs, self.nprob, ctypes.byref(io), _ptr(self.ws), self.ws.numel(),
                                        _stream()), "bo_wide_gauss_loss")


# ------------------------------------------------------------- graph GMRFs

def rcm(indptr, indices):
    """Reverse Cuthill-McKee ordering of a symmetric CSR pattern (host, see
    bo_rcm).  Returns (perm, iperm, bandwidth): perm[new] = old."""
    import numpy as np
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    n = ip.size - 1
    perm = np.zeros(max(n, 1), dtype=np.int64)
    iperm = np.zeros(max(n, 1), dtype=np.int64)
    bw = ctypes.c_int64(0)
    hp = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(lib().bo_rcm(n, hp(ip), hp(ix), hp(perm), hp(iperm), ctypes.byref(bw)), "bo_rcm")
    return perm[:n], iperm[:n], int(bw.value)


def csr_permute(indptr, indices, perm, iperm):
    """The pattern of P Q P^T (host, see bo_csr_permute): (indptr, indices,
    map) with new entry e' taken from Q's entry map[e']."""
    import numpy as np
    ip = np.ascontiguousarray(indptr, dtype=np.int64)
    ix = np.ascontiguousarray(indices, dtype=np.int64)
    pm = np.ascontiguousarray(perm, dtype=np.int64)
    ipm = np.ascontiguousarray(iperm, dtype=np.int64)
    n = ip.size - 1
    oip = np.zeros(n + 1, dtype=np.int64)
    oix = np.zeros(max(ix.size, 1), dtype=np.int64)
    mp = np.zeros(max(ix.size, 1), dtype=np.int64)
    hp = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(lib().bo_csr_permute(n, hp(ip), hp(ix), hp(pm), hp(ipm), hp(oip), hp(oix), hp(mp)), "bo_csr_permute")
    return oip, oix[:ix.size], mp[:ix.size]


def csr_to_band(prec: int, indptr, indices, vals, k: int, band, diag=None, dropped=None, nsets: int = 1):
    """Lower bands of a symmetric CSR matrix whose rows are in band order, for
    nsets value sets (device tensors, see bo_csr_to_band).  Returns the device
    int64 count of dropped entries."""
    n = indptr.numel() - 1
    if dropped is None:
        dropped = torch.zeros(1, dtype=torch.int64, device=indptr.device)
    _check(lib().bo_csr_to_band(prec, n, nsets, _ptr(indptr), _ptr(indices), indices.numel(), _ptr(vals), k, k + 1,
                                _ptr(band), _ptr(diag), _ptr(dropped), _stream()), "bo_csr_to_band")
    return dropped


def band_to_csr_grad(prec: int, indptr, indices, k: int, gband, gdiag, gvals, nsets: int = 1):
    """Gradient with respect to the CSR entries from the band gradient for
    nsets value sets (device tensors, see bo_band_to_csr_grad)."""
    n = indptr.numel() - 1
    _check(lib().bo_band_to_csr_grad(prec, n, nsets, _ptr(indptr), _ptr(indices), indices.numel(), k, k + 1,
                                     _ptr(gband), _ptr(gdiag), _ptr(gvals), _stream()), "bo_band_to_csr_grad")
