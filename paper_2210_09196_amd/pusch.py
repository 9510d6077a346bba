"""Python binding of libpusch.so (include/pusch.h) for torch device tensors.

Argument marshalling only: every stage runs in the library's HIP kernels on
the caller's current torch stream.  There is no fallback path -- if the shared
library is missing or fails to load, every call raises.  Calls with an empty
batch return their (empty) outputs without entering the library, since torch
gives empty tensors a null data pointer.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpusch.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pusch.h")

MAX_PILOTS = 4
CELLS_MIXED, CELLS_STREAMS = 1, 2  # pusch_cells flags


def cells_with_plan(p: int) -> int:
    """pusch_cells flag that runs launch plan p (PUSCH_CELLS_WITH_PLAN)."""
    return 4 | (p << 3)
SLOT_STAGES = ("fft", "beamform", "chest", "mmse")


class PuschError(RuntimeError):
    """A libpusch call returned a negative status code."""


class SlotDesc(ctypes.Structure):
    _fields_ = [
        ("n_ant", ctypes.c_int),
        ("n_fft", ctypes.c_int),
        ("n_sc", ctypes.c_int),
        ("n_symb", ctypes.c_int),
        ("n_beams", ctypes.c_int),
        ("n_ue", ctypes.c_int),
        ("n_pilot", ctypes.c_int),
        ("pilot_symb", ctypes.c_int * MAX_PILOTS),
        ("sigma2", ctypes.c_float),
        ("W", ctypes.c_void_p),
        ("pilots", ctypes.c_void_p),
        ("noise_est", ctypes.c_int),
        ("sigma2_est", ctypes.c_void_p),
        ("refine", ctypes.c_int),
        ("time_varying", ctypes.c_int),
        ("comb_aligned", ctypes.c_int),
        ("fft_mfma", ctypes.c_int),
    ]


_lib = None
class CellsPlan(ctypes.Structure):
    _fields_ = [("fft_merged", ctypes.c_int), ("bf_merged", ctypes.c_int), ("mmse_merged", ctypes.c_int)]


CELLS_PLANS = 8

_P = ctypes.c_void_p
_I = ctypes.c_int
_LL = ctypes.c_longlong
_F = ctypes.c_float
_SIG = {
    "pusch_strerror": (ctypes.c_char_p, [_I]),
    "pusch_init": (_I, []),
    "pusch_fft": (_I, [_P, _P, _I, _I, _LL, _P]),
    "pusch_beamform": (_I, [_P, _P, _P, _I, _I, _I, _LL, _LL, _P]),
    "pusch_chest": (_I, [_P, _P, _P, _I, _I, _I, _I, _LL, _P]),
    "pusch_noise_est_workspace_bytes": (ctypes.c_size_t, [_LL]),
    "pusch_noise_est": (_I, [_P, _P, _P, _I, _I, _I, _I, _LL, _P, ctypes.c_size_t, _P]),
    "pusch_noise_est_static": (_I, [_P, _P, _P, _I, _I, _I, _I, _LL, _P]),
    "pusch_mmse_solve": (_I, [_P, _P, _F, _P, _I, _I, _I, _I, _LL, _P, _P]),
    "pusch_slot_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SlotDesc), _LL]),
    "pusch_slot": (_I, [ctypes.POINTER(SlotDesc), _LL, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "pusch_slot_mixed_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SlotDesc), _LL]),
    "pusch_slot_mixed": (_I, [ctypes.POINTER(SlotDesc), _LL, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "pusch_slot_bf16_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SlotDesc), _LL]),
    "pusch_slot_bf16": (_I, [ctypes.POINTER(SlotDesc), _LL, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "pusch_cells_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SlotDesc), _I, ctypes.POINTER(_LL), _I]),
    "pusch_cells": (_I, [ctypes.POINTER(SlotDesc), _I, ctypes.POINTER(_LL), ctypes.POINTER(_P), ctypes.POINTER(_P),
                         ctypes.POINTER(_P), _P, ctypes.c_size_t, _I, _P]),
    "pusch_cells_tune": (_I, [ctypes.POINTER(SlotDesc), _I, ctypes.POINTER(_LL), ctypes.POINTER(_P),
                              ctypes.POINTER(_P), ctypes.POINTER(_P), _P, ctypes.c_size_t, _I, _I,
                              ctypes.POINTER(CellsPlan), ctypes.POINTER(_F), _I, _P]),
    "pusch_cells_plan_get": (_I, [ctypes.POINTER(SlotDesc), _I, ctypes.POINTER(_LL), _I, ctypes.POINTER(CellsPlan)]),
    "pusch_dn_workspace_bytes": (ctypes.c_size_t, [_I, _I, _LL]),
    "pusch_dn_ls_grid": (_I, [_P, _P, _P, _I, _I, _I, _I, _I, ctypes.POINTER(_I), _LL, _P]),
    "pusch_dn_forward": (_I, [_P, _P, _P, _F, _I, _I, _LL, _P, ctypes.c_size_t, _P]),
    "pusch_dn_backward": (_I, [_P, _P, _P, _P, _I, _I, _LL, _P, ctypes.c_size_t, _P]),
    "pusch_dn_loss": (_I, [_P, _P, _P, _P, _P, _I, _I, _LL, _P, ctypes.c_size_t, _P]),
    "pusch_dn_adam": (_I, [_P, _P, _P, _P, _I, _F, _F, _F, _F, _P]),
    "pusch_slot_denoised_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SlotDesc), _LL]),
    "pusch_slot_denoised": (_I, [ctypes.POINTER(SlotDesc), _LL, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "pusch_profile_begin": (_I, [_I]),
    "pusch_profile_end": (_I, [ctypes.POINTER(_F), _I]),
}


def header_symbols(path: str = HEADER) -> list[str]:
    """Names of the functions include/pusch.h declares."""
    text = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int|size_t)\s+(pusch_\w+)\s*\(", text, re.M)))


def lib() -> ctypes.CDLL:
    """Load libpusch.so once and attach the C signatures; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PuschError(f"{LIB_PATH} is not built; run `python -m paper_2210_09196_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def strerror(code: int) -> str:
    return lib().pusch_strerror(int(code)).decode()


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise PuschError(f"{what}: {strerror(rc)} ({rc})")
    return rc


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _c64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise PuschError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.complex64:
        raise PuschError(f"{name} must be complex64, got {t.dtype}")
    if not t.is_contiguous():
        raise PuschError(f"{name} must be contiguous")
    return t


def _sized(t, n: int, dtype, name: str) -> torch.Tensor:
    """An output buffer the library writes n elements of dtype into: a contiguous device tensor of exactly n."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise PuschError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise PuschError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise PuschError(f"{name} must be contiguous")
    if t.numel() != n:
        raise PuschError(f"{name} must hold {n} elements, got {t.numel()}")
    return t


def _status(status, n_items: int, n_sc: int, device, name: str = "status"):
    """status=True: a new [n_items, n_sc] int32 tensor; False/None: no flags; else a caller tensor of that size."""
    if status is True:
        return torch.empty(n_items, n_sc, dtype=torch.int32, device=device)
    if status is False or status is None:
        return None
    return _sized(status, n_items * n_sc, torch.int32, name)


def _beamformer(W, n_beams: int, n_ant: int, name: str) -> torch.Tensor:
    """A caller-supplied beamformer: the library reads n_beams * n_ant values from it, so its shape
    must be exactly [n_beams, n_ant]."""
    _c64(W, name)
    if tuple(W.shape) != (n_beams, n_ant):
        raise PuschError(f"{name} must be [{n_beams}, {n_ant}], got {list(W.shape)}")
    return W


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def init() -> None:
    _check(lib().pusch_init(), "pusch_init")


def fft(x: torch.Tensor, n_sc: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Unscaled forward FFT over the last axis; n_sc > 0 keeps the centred active bins."""
    _c64(x, "x")
    n_fft = x.shape[-1]
    batch = x.numel() // n_fft if n_fft else 0
    out_len = n_sc if n_sc else n_fft
    if out is None:
        out = torch.empty(*x.shape[:-1], out_len, dtype=torch.complex64, device=x.device)
    _c64(out, "out")
    if out.numel() != batch * out_len:
        raise PuschError("fft: output has the wrong size")
    if batch == 0:
        return out
    _check(lib().pusch_fft(x.data_ptr(), out.data_ptr(), n_fft, n_sc, batch, _stream()), "pusch_fft")
    return out


def beamform(X: torch.Tensor, n_beams: int, W: torch.Tensor | None = None, n_re: int | None = None,
             out: torch.Tensor | None = None) -> torch.Tensor:
    """Y[i, n, b] = sum_a W[b, a] X[i, a, n] for X [batch, n_ant, ld_x]; returns [batch, n_re, n_beams]."""
    _c64(X, "X")
    if X.dim() == 2:
        X = X.unsqueeze(0)
    batch, n_ant, ld_x = X.shape
    n_re = ld_x if n_re is None else n_re
    if W is not None:
        _c64(W, "W")
        if tuple(W.shape) != (n_beams, n_ant):
            raise PuschError("beamform: W must be [n_beams, n_ant]")
    if out is None:
        out = torch.empty(batch, n_re, n_beams, dtype=torch.complex64, device=X.device)
    _sized(out, batch * n_re * n_beams, torch.complex64, "out")
    if batch == 0 or n_re == 0:
        return out
    _check(lib().pusch_beamform(_ptr(W), X.data_ptr(), out.data_ptr(), n_beams, n_ant, n_re, ld_x, batch, _stream()),
           "pusch_beamform")
    return out


def chest(Yp: torch.Tensor, pilots: torch.Tensor, n_ue: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """LS channel estimate: Yp [batch, n_pilot, n_sc, n_beams], pilots [batch, n_pilot, n_sc]
    -> H [batch, n_sc, n_ue, n_beams]."""
    _c64(Yp, "Yp")
    _c64(pilots, "pilots")
    batch, n_pilot, n_sc, n_beams = Yp.shape
    if tuple(pilots.shape) != (batch, n_pilot, n_sc):
        raise PuschError("chest: pilots must be [batch, n_pilot, n_sc]")
    if out is None:
        out = torch.empty(batch, n_sc, n_ue, n_beams, dtype=torch.complex64, device=Yp.device)
    _sized(out, batch * n_sc * n_ue * n_beams, torch.complex64, "out")
    if batch == 0:
        return out
    _check(lib().pusch_chest(Yp.data_ptr(), pilots.data_ptr(), out.data_ptr(), n_beams, n_ue, n_sc, n_pilot, batch,
                             _stream()), "pusch_chest")
    return out


def noise_est(Yp: torch.Tensor, pilots: torch.Tensor, n_ue: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Noise variance per batch item from the pilot symbols: Yp [batch, n_pilot, n_sc, n_beams],
    pilots [batch, n_pilot, n_sc] -> sigma2 [batch] float32."""
    _c64(Yp, "Yp")
    _c64(pilots, "pilots")
    batch, n_pilot, n_sc, n_beams = Yp.shape
    if tuple(pilots.shape) != (batch, n_pilot, n_sc):
        raise PuschError("noise_est: pilots must be [batch, n_pilot, n_sc]")
    if out is None:
        out = torch.empty(batch, dtype=torch.float32, device=Yp.device)
    _sized(out, batch, torch.float32, "out")
    if batch == 0:
        return out
    nbytes = int(lib().pusch_noise_est_workspace_bytes(batch))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=Yp.device)
    _check(lib().pusch_noise_est(Yp.data_ptr(), pilots.data_ptr(), out.data_ptr(), n_beams, n_ue, n_sc, n_pilot, batch,
                                 ws.data_ptr(), nbytes, _stream()), "pusch_noise_est")
    return out


NOISE_EST_STATIC_MAX_BATCH = 1024


def noise_est_static(Yp: torch.Tensor, pilots: torch.Tensor, n_ue: int, out: torch.Tensor | None = None
                     ) -> torch.Tensor:
    """As noise_est, through pusch_noise_est_static: no workspace, the library's own device scratch
    (at most NOISE_EST_STATIC_MAX_BATCH items per call; calls that overlap on one GPU race)."""
    _c64(Yp, "Yp")
    _c64(pilots, "pilots")
    batch, n_pilot, n_sc, n_beams = Yp.shape
    if tuple(pilots.shape) != (batch, n_pilot, n_sc):
        raise PuschError("noise_est_static: pilots must be [batch, n_pilot, n_sc]")
    if batch > NOISE_EST_STATIC_MAX_BATCH:
        raise PuschError(f"noise_est_static: at most {NOISE_EST_STATIC_MAX_BATCH} items per call, got {batch}")
    if out is None:
        out = torch.empty(batch, dtype=torch.float32, device=Yp.device)
    _sized(out, batch, torch.float32, "out")
    if batch == 0:
        return out
    _check(lib().pusch_noise_est_static(Yp.data_ptr(), pilots.data_ptr(), out.data_ptr(), n_beams, n_ue, n_sc,
                                        n_pilot, batch, _stream()), "pusch_noise_est_static")
    return out


def mmse_solve(H: torch.Tensor, Yd: torch.Tensor, sigma2: float, out: torch.Tensor | None = None,
               status: torch.Tensor | None | bool = True):
    """MMSE detection: H [batch, n_sc, n_ue, n_beams], Yd [batch, n_data, n_sc, n_beams]
    -> (x_hat [batch, n_data, n_sc, n_ue], status [batch, n_sc] int32 or None)."""
    _c64(H, "H")
    _c64(Yd, "Yd")
    batch, n_sc, n_ue, n_beams = H.shape
    if Yd.dim() != 4 or Yd.shape[0] != batch or Yd.shape[2] != n_sc or Yd.shape[3] != n_beams:
        raise PuschError("mmse_solve: Yd must be [batch, n_data, n_sc, n_beams]")
    n_data = Yd.shape[1]
    if out is None:
        out = torch.empty(batch, n_data, n_sc, n_ue, dtype=torch.complex64, device=H.device)
    _sized(out, batch * n_data * n_sc * n_ue, torch.complex64, "out")
    status = _status(status, batch, n_sc, H.device)
    if batch == 0 or n_sc == 0:
        return out, status
    _check(lib().pusch_mmse_solve(H.data_ptr(), Yd.data_ptr(), float(sigma2), out.data_ptr(), n_beams, n_ue, n_sc,
                                  n_data, batch, _ptr(status), _stream()), "pusch_mmse_solve")
    return out, status


class Slot:
    """A fixed slot geometry with its device workspace, for repeated pusch_slot calls.

    precision="mixed" uses pusch_slot_mixed (FP16 active-bin grids between
    OFDM demodulation and beamforming, beamforming on FP16 matrix cores with
    FP32 accumulation, FP32 estimation and detection); precision="bf16" uses
    pusch_slot_bf16 (the same with bfloat16 grids and BF16 matrix cores).  sigma2=None estimates
    every slot's noise variance from its pilot symbols; each call leaves the
    estimates in self.sigma2_est ([n_slot] float32).  refine=True adds one
    iterative-refinement step to the MIMO solve.  time_varying=True gives
    every data symbol its own channel estimate (interpolated in time between
    the pilot symbols) and its own factorisation.  comb_aligned=True: the
    pilot comb without stagger (each UE on the same subcarriers in every pilot
    symbol).  fft_mfma=True (with precision "mixed" or "bf16", n_fft 4096):
    the FFT's radix-16 passes on the matrix cores."""

    def __init__(self, n_ant: int, n_fft: int, n_sc: int, n_symb: int, n_beams: int, n_ue: int, pilot_symb,
                 sigma2: float | None, n_slot: int, W: torch.Tensor | None = None, device="cuda",
                 precision: str = "fp32", refine: bool = False, time_varying: bool = False,
                 comb_aligned: bool = False, fft_mfma: bool = False):
        if precision not in ("fp32", "mixed", "bf16"):
            raise PuschError("precision is 'fp32', 'mixed' or 'bf16'")
        self.precision = precision
        self.mixed = precision == "mixed"
        pilot_symb = list(pilot_symb)
        if not 1 <= len(pilot_symb) <= MAX_PILOTS:
            raise PuschError("1..4 pilot symbols")
        self.desc = SlotDesc()
        d = self.desc
        d.n_ant, d.n_fft, d.n_sc, d.n_symb = n_ant, n_fft, n_sc, n_symb
        d.n_beams, d.n_ue, d.n_pilot = n_beams, n_ue, len(pilot_symb)
        for j, s in enumerate(pilot_symb):
            d.pilot_symb[j] = s
        self.sigma2_est = _noise_fields(d, sigma2, n_slot, device)
        d.refine = 1 if refine else 0
        d.time_varying = 1 if time_varying else 0
        d.comb_aligned = 1 if comb_aligned else 0
        d.fft_mfma = 1 if fft_mfma else 0
        self.W = None if W is None else _beamformer(W, n_beams, n_ant, "W")
        d.W = _ptr(self.W)
        self.n_slot = n_slot
        self.n_data = n_symb - len(pilot_symb)
        wsb = {"fp32": lib().pusch_slot_workspace_bytes, "mixed": lib().pusch_slot_mixed_workspace_bytes,
               "bf16": lib().pusch_slot_bf16_workspace_bytes}[precision]
        nbytes = wsb(ctypes.byref(d), n_slot)
        if nbytes == 0 and n_slot > 0:
            raise PuschError("the library rejected the slot geometry (workspace size 0)")
        self.ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        self.ws_bytes = int(nbytes)

    def __call__(self, x_td: torch.Tensor, pilots: torch.Tensor, x_hat: torch.Tensor | None = None,
                 status: torch.Tensor | None | bool = True):
        d = self.desc
        _c64(x_td, "x_td")
        _c64(pilots, "pilots")
        if tuple(x_td.shape) != (self.n_slot, d.n_symb, d.n_ant, d.n_fft):
            raise PuschError(f"x_td must be [{self.n_slot}, {d.n_symb}, {d.n_ant}, {d.n_fft}]")
        if tuple(pilots.shape) != (self.n_slot, d.n_pilot, d.n_sc):
            raise PuschError(f"pilots must be [{self.n_slot}, {d.n_pilot}, {d.n_sc}]")
        if x_hat is None:
            x_hat = torch.empty(self.n_slot, self.n_data, d.n_sc, d.n_ue, dtype=torch.complex64, device=x_td.device)
        _sized(x_hat, self.n_slot * self.n_data * d.n_sc * d.n_ue, torch.complex64, "x_hat")
        status = _status(status, self.n_slot, d.n_sc, x_td.device)
        if self.n_slot == 0:
            return x_hat, status
        d.pilots = pilots.data_ptr()
        name = {"fp32": "pusch_slot", "mixed": "pusch_slot_mixed", "bf16": "pusch_slot_bf16"}[self.precision]
        fn = getattr(lib(), name)
        _check(fn(ctypes.byref(d), self.n_slot, x_td.data_ptr(), x_hat.data_ptr(), _ptr(status), self.ws.data_ptr(),
                  self.ws_bytes, _stream()), name)
        return x_hat, status


def _noise_fields(d: SlotDesc, sigma2, n_slot: int, device) -> torch.Tensor | None:
    """sigma2 None: estimate it per slot (noise_est) into a new [n_slot] float32 tensor, returned."""
    if sigma2 is None:
        est = torch.zeros(max(int(n_slot), 1), dtype=torch.float32, device=device)
        d.sigma2, d.noise_est, d.sigma2_est = 0.0, 1, est.data_ptr()
        return est
    d.sigma2, d.noise_est, d.sigma2_est = float(sigma2), 0, None
    return None


def _fill_desc(d: SlotDesc, n_ant, n_fft, n_sc, n_symb, n_beams, n_ue, pilot_symb, sigma2, W, n_slot=1,
               device="cuda") -> torch.Tensor | None:
    pilot_symb = list(pilot_symb)
    if not 1 <= len(pilot_symb) <= MAX_PILOTS:
        raise PuschError("1..4 pilot symbols")
    d.n_ant, d.n_fft, d.n_sc, d.n_symb = n_ant, n_fft, n_sc, n_symb
    d.n_beams, d.n_ue, d.n_pilot = n_beams, n_ue, len(pilot_symb)
    for j, s in enumerate(pilot_symb):
        d.pilot_symb[j] = s
    d.W = _ptr(W)
    return _noise_fields(d, sigma2, n_slot, device)


class Cells:
    """Independent cells of different slot geometries, run by one pusch_cells call.

    Each cell is a dict with the slot geometry (n_ant, n_fft, n_sc, n_symb,
    n_beams, n_ue, pilot_symb), sigma2 (None: estimated per slot, left in
    self.sigma2_est[c]), n_slot (>= 1) and optionally W, refine,
    time_varying and comb_aligned.  The workspace is allocated once here.  A call runs the
    cells the grouped kernels take as one launch per stage and kernel shape on
    the current torch stream, and the others on the library's side streams,
    forked from and joined back to that stream, so it can be captured into a
    HIP graph; grouped=False runs every cell on the side streams, and plan=p
    fixes the grouped cells' launch plan (else the one pusch_cells_tune
    recorded for the cell set, or the default).
    """

    def __init__(self, cells: list[dict], device="cuda", precision: str = "fp32", grouped: bool = True,
                 plan: int | None = None):
        if precision not in ("fp32", "mixed"):
            raise PuschError("precision is 'fp32' or 'mixed'")
        if plan is not None and not 0 <= plan < CELLS_PLANS:
            raise PuschError(f"plan is 0..{CELLS_PLANS - 1}")
        self.flags = (CELLS_MIXED if precision == "mixed" else 0) | (0 if grouped else CELLS_STREAMS) | \
            (0 if plan is None else cells_with_plan(plan))
        n = len(cells)
        if n < 1:
            raise PuschError("at least one cell")
        self.n = n
        self.descs = (SlotDesc * n)()
        self.n_slot = (_LL * n)()
        self.W = []
        self.geom = []
        self.sigma2_est = []
        for c, g in enumerate(cells):
            if int(g["n_slot"]) < 1:
                raise PuschError("every cell needs n_slot >= 1")
            W = g.get("W")
            W = None if W is None else _beamformer(W, g["n_beams"], g["n_ant"], f"cell {c}: W")
            self.W.append(W)
            self.sigma2_est.append(
                _fill_desc(self.descs[c], g["n_ant"], g["n_fft"], g["n_sc"], g["n_symb"], g["n_beams"], g["n_ue"],
                           g["pilot_symb"], g["sigma2"], W, int(g["n_slot"]), device))
            self.descs[c].refine = 1 if g.get("refine") else 0
            self.descs[c].time_varying = 1 if g.get("time_varying") else 0
            self.descs[c].comb_aligned = 1 if g.get("comb_aligned") else 0
            self.n_slot[c] = int(g["n_slot"])
            self.geom.append(dict(g))
        nbytes = lib().pusch_cells_workspace_bytes(self.descs, n, self.n_slot, self.flags)
        if nbytes == 0:
            raise PuschError("pusch_cells_workspace_bytes rejected a cell geometry")
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.ws_bytes = int(nbytes)

    def outputs(self, device="cuda"):
        """Fresh (x_hat, status) tensors for every cell."""
        xs, st = [], []
        for c in range(self.n):
            d = self.descs[c]
            xs.append(torch.empty(self.n_slot[c], d.n_symb - d.n_pilot, d.n_sc, d.n_ue, dtype=torch.complex64,
                                  device=device))
            st.append(torch.empty(self.n_slot[c], d.n_sc, dtype=torch.int32, device=device))
        return xs, st

    def __call__(self, x_tds, pilots, x_hats=None, statuses=None):
        args, x_hats, statuses = self._args(x_tds, pilots, x_hats, statuses)
        _check(lib().pusch_cells(*args, _stream()), "pusch_cells")
        return x_hats, statuses

    def tune(self, x_tds, pilots, reps: int = 5, x_hats=None, statuses=None):
        """pusch_cells_tune: times every launch plan on these inputs and records the fastest for
        this cell set; returns (plan dict, median us of plan p for p in 0..7)."""
        args, x_hats, statuses = self._args(x_tds, pilots, x_hats, statuses)
        plan = CellsPlan()
        us = (_F * CELLS_PLANS)()
        _check(lib().pusch_cells_tune(*args, int(reps), ctypes.byref(plan), us, CELLS_PLANS, _stream()),
               "pusch_cells_tune")
        return _plan_dict(plan), [float(v) for v in us]

    def plan(self):
        """(plan dict, tuned) that pusch_cells uses for this cell set."""
        plan = CellsPlan()
        rc = lib().pusch_cells_plan_get(self.descs, self.n, self.n_slot, self.flags, ctypes.byref(plan))
        if rc < 0:
            _check(rc, "pusch_cells_plan_get")
        return _plan_dict(plan), bool(rc)

    def _args(self, x_tds, pilots, x_hats, statuses):
        if len(x_tds) != self.n or len(pilots) != self.n:
            raise PuschError(f"{self.n} x_td and pilots tensors expected")
        if x_hats is None:
            x_hats, statuses = self.outputs(x_tds[0].device)
        if len(x_hats) != self.n or (statuses is not None and len(statuses) != self.n):
            raise PuschError(f"{self.n} x_hat (and status) tensors expected")
        for c in range(self.n):
            d = self.descs[c]
            _c64(x_tds[c], "x_td")
            _c64(pilots[c], "pilots")
            _c64(x_hats[c], "x_hat")
            ns = self.n_slot[c]
            if tuple(x_tds[c].shape) != (ns, d.n_symb, d.n_ant, d.n_fft):
                raise PuschError(f"cell {c}: x_td must be [{ns}, {d.n_symb}, {d.n_ant}, {d.n_fft}]")
            if tuple(pilots[c].shape) != (ns, d.n_pilot, d.n_sc):
                raise PuschError(f"cell {c}: pilots must be [{ns}, {d.n_pilot}, {d.n_sc}]")
            if tuple(x_hats[c].shape) != (ns, d.n_symb - d.n_pilot, d.n_sc, d.n_ue):
                raise PuschError(f"cell {c}: x_hat has the wrong shape")
            if statuses is not None and statuses[c] is not None:
                _sized(statuses[c], ns * d.n_sc, torch.int32, f"cell {c}: status")
            d.pilots = pilots[c].data_ptr()
        xp = (_P * self.n)(*[t.data_ptr() for t in x_tds])
        op = (_P * self.n)(*[t.data_ptr() for t in x_hats])
        sp = None if statuses is None else (_P * self.n)(*[_ptr(t) for t in statuses])
        self._keep = (xp, op, sp)
        return (self.descs, self.n, self.n_slot, xp, op, sp, self.ws.data_ptr(), self.ws_bytes, self.flags), \
            x_hats, statuses


def _plan_dict(plan: CellsPlan) -> dict:
    return {"fft_merged": bool(plan.fft_merged), "bf_merged": bool(plan.bf_merged),
            "mmse_merged": bool(plan.mmse_merged)}


def profile_begin(max_calls: int) -> None:
    _check(lib().pusch_profile_begin(int(max_calls)), "pusch_profile_begin")


def profile_end() -> tuple[int, dict]:
    """Returns (calls recorded, {stage: summed device ms})."""
    buf = (ctypes.c_float * len(SLOT_STAGES))()
    calls = _check(lib().pusch_profile_end(buf, len(SLOT_STAGES)), "pusch_profile_end")
    return calls, {name: float(buf[i]) for i, name in enumerate(SLOT_STAGES)}


# ----------------------------------------------------------------------------- LS-estimate denoiser

DN_PARAMS = 19682


def _f32(t, n, name):
    return _sized(t, n, torch.float32, name)


def dn_ls_grid(Yp: torch.Tensor, pilots: torch.Tensor, n_ue: int, n_symb: int, pilot_symb,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """LS estimate on every symbol: Yp [batch, n_pilot, n_sc, n_beams], pilots [batch, n_pilot, n_sc]
    -> grid [batch, n_ue, n_beams, n_symb, n_sc]."""
    _c64(Yp, "Yp")
    _c64(pilots, "pilots")
    batch, n_pilot, n_sc, n_beams = Yp.shape
    if tuple(pilots.shape) != (batch, n_pilot, n_sc):
        raise PuschError("dn_ls_grid: pilots must be [batch, n_pilot, n_sc]")
    ps = list(pilot_symb)
    if len(ps) != n_pilot:
        raise PuschError("dn_ls_grid: one symbol index per pilot symbol")
    if out is None:
        out = torch.empty(batch, n_ue, n_beams, n_symb, n_sc, dtype=torch.complex64, device=Yp.device)
    _sized(out, batch * n_ue * n_beams * n_symb * n_sc, torch.complex64, "out")
    if batch == 0:
        return out
    arr = (_I * n_pilot)(*ps)
    _check(lib().pusch_dn_ls_grid(Yp.data_ptr(), pilots.data_ptr(), out.data_ptr(), n_beams, n_ue, n_sc, n_symb,
                                  n_pilot, arr, batch, _stream()), "pusch_dn_ls_grid")
    return out


class Denoiser:
    """Workspace for running and training the LS-estimate denoiser on n_grid grids of n_symb x n_sc
    (complex [n_grid, n_symb, n_sc]).  Parameters are a float32 tensor of DN_PARAMS values."""

    def __init__(self, n_symb: int, n_sc: int, n_grid: int, device="cuda"):
        nbytes = int(lib().pusch_dn_workspace_bytes(n_symb, n_sc, n_grid))
        if nbytes == 0:
            raise PuschError("pusch_dn_workspace_bytes rejected the grid shape")
        self.n_symb, self.n_sc, self.n_grid = n_symb, n_sc, n_grid
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.ws_bytes = nbytes
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=device)

    def _grid(self, t, name):
        return _sized(t, self.n_grid * self.n_symb * self.n_sc, torch.complex64, name)

    def forward(self, params: torch.Tensor, grid: torch.Tensor, out: torch.Tensor | None = None,
                sigma: float = 1.0) -> torch.Tensor:
        """out = grid + sigma net(grid / sigma); sigma = 1 (the default) is the plain network."""
        _f32(params, DN_PARAMS, "params")
        self._grid(grid, "grid")
        if out is None:
            out = torch.empty_like(grid)
        self._grid(out, "out")
        if self.n_grid == 0:
            return out
        _check(lib().pusch_dn_forward(params.data_ptr(), grid.data_ptr(), out.data_ptr(), float(sigma), self.n_symb,
                                      self.n_sc, self.n_grid, self.ws.data_ptr(), self.ws_bytes, _stream()),
               "pusch_dn_forward")
        return out

    def loss(self, out: torch.Tensor, target: torch.Tensor, dout: torch.Tensor | None = None,
             weights: torch.Tensor | None = None):
        """(loss [1] float32 on the device, dout = dL/d(out)); weights: one float32 per grid, or None."""
        self._grid(out, "out")
        self._grid(target, "target")
        if dout is None:
            dout = torch.empty_like(out)
        self._grid(dout, "dout")
        if weights is not None:
            _f32(weights, self.n_grid, "weights")
        _check(lib().pusch_dn_loss(out.data_ptr(), target.data_ptr(), _ptr(weights), dout.data_ptr(),
                                   self.loss_buf.data_ptr(), self.n_symb, self.n_sc, self.n_grid, self.ws.data_ptr(),
                                   self.ws_bytes, _stream()), "pusch_dn_loss")
        return self.loss_buf, dout

    def backward(self, params: torch.Tensor, grid: torch.Tensor, dout: torch.Tensor,
                 grads: torch.Tensor | None = None) -> torch.Tensor:
        _f32(params, DN_PARAMS, "params")
        self._grid(grid, "grid")
        self._grid(dout, "dout")
        if grads is None:
            grads = torch.empty(DN_PARAMS, dtype=torch.float32, device=params.device)
        _f32(grads, DN_PARAMS, "grads")
        _check(lib().pusch_dn_backward(params.data_ptr(), grid.data_ptr(), dout.data_ptr(), grads.data_ptr(),
                                       self.n_symb, self.n_sc, self.n_grid, self.ws.data_ptr(), self.ws_bytes,
                                       _stream()), "pusch_dn_backward")
        return grads


def dn_adam(params: torch.Tensor, grads: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
            beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    for t, name in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
        _f32(t, DN_PARAMS, name)
    _check(lib().pusch_dn_adam(params.data_ptr(), grads.data_ptr(), m.data_ptr(), v.data_ptr(), int(step), float(lr),
                               float(beta1), float(beta2), float(eps), _stream()), "pusch_dn_adam")


class DenoisedSlot:
    """The receive chain with the denoised LS estimate and the LS fallback (pusch_slot_denoised) for a
    fixed slot geometry; each call returns (x_hat, status, used_dn [n_slot] int32)."""

    def __init__(self, n_ant: int, n_fft: int, n_sc: int, n_symb: int, n_beams: int, n_ue: int, pilot_symb,
                 sigma2: float, n_slot: int, W: torch.Tensor | None = None, device="cuda"):
        pilot_symb = list(pilot_symb)
        self.desc = SlotDesc()
        d = self.desc
        _fill_desc(d, n_ant, n_fft, n_sc, n_symb, n_beams, n_ue, pilot_symb, sigma2, W, n_slot, device)
        if sigma2 is None:
            raise PuschError("the denoised chain takes sigma2 as given")
        self.W = None if W is None else _beamformer(W, n_beams, n_ant, "W")
        d.W = _ptr(self.W)
        self.n_slot = n_slot
        self.n_data = n_symb - len(pilot_symb)
        nbytes = lib().pusch_slot_denoised_workspace_bytes(ctypes.byref(d), n_slot)
        if nbytes == 0 and n_slot > 0:
            raise PuschError("the library rejected the slot geometry (workspace size 0)")
        self.ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        self.ws_bytes = int(nbytes)

    def __call__(self, x_td: torch.Tensor, pilots: torch.Tensor, params: torch.Tensor):
        d = self.desc
        _c64(x_td, "x_td")
        _c64(pilots, "pilots")
        _f32(params, DN_PARAMS, "params")
        if tuple(x_td.shape) != (self.n_slot, d.n_symb, d.n_ant, d.n_fft):
            raise PuschError(f"x_td must be [{self.n_slot}, {d.n_symb}, {d.n_ant}, {d.n_fft}]")
        if tuple(pilots.shape) != (self.n_slot, d.n_pilot, d.n_sc):
            raise PuschError(f"pilots must be [{self.n_slot}, {d.n_pilot}, {d.n_sc}]")
        x_hat = torch.empty(self.n_slot, self.n_data, d.n_sc, d.n_ue, dtype=torch.complex64, device=x_td.device)
        status = torch.empty(self.n_slot, d.n_sc, dtype=torch.int32, device=x_td.device)
        used = torch.empty(self.n_slot, dtype=torch.int32, device=x_td.device)
        if self.n_slot == 0:
            return x_hat, status, used
        d.pilots = pilots.data_ptr()
        _check(lib().pusch_slot_denoised(ctypes.byref(d), self.n_slot, x_td.data_ptr(), params.data_ptr(),
                                         x_hat.data_ptr(), status.data_ptr(), used.data_ptr(), self.ws.data_ptr(),
                                         self.ws_bytes, _stream()), "pusch_slot_denoised")
        return x_hat, status, used
