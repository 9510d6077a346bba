"""Seeded synthetic PUSCH slots: transmitter, channel and noise.

This module produces the inputs that both the HIP receive chain and its FP64
CPU oracle consume, so that both sides see exactly the same samples.  It models
the uplink of Sec. II: N_L UEs send QAM data and pilots on an OFDM grid of
N_SC subcarriers x N_symb symbols (the block-type pilot arrangement, whole OFDM
symbols of pilots), the signal passes a multi-antenna channel and picks up
additive white Gaussian noise (the signal model y = Hx + n of Eq. 1, applied
per antenna before beamforming), and the receiver gets one time-domain OFDM
symbol per antenna (inverse FFT of the grid, no cyclic prefix).

It holds none of the receiver's arithmetic: no FFT demodulation, beamforming,
channel estimation or detection lives here.  Readings where the paper is silent:

* subcarrier placement: active subcarrier k sits on FFT bin (k - N_act//2) mod N
  (centred band, DC used);
* pilots of the N_L UEs share one pilot symbol as a frequency comb: on pilot
  symbol j (0-based among the pilot symbols) subcarrier k carries the pilot of
  UE (k + o_j) mod N_L, with o_j = j * (N_L // N_pilot), all other UEs send 0
  there;
* QAM symbols use the Gray mappings of 3GPP TS 38.211 Sec. 5.1 with unit
  average energy; pilots are QPSK;
* channel: frequency-flat i.i.d. CN(0,1) (one N_R x N_L matrix), or an 8-tap
  tapped-delay-line with exponential power-delay profile P_t ~ exp(-t),
  uniform tap spacing chosen so the RMS delay spread equals the target;
* SNR = 1/sigma^2 per receive antenna per UE (unit-energy symbols, unit-power
  channel); time-domain noise CN(0, sigma^2/N) so each FFT bin carries
  CN(0, sigma^2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "SlotConfig",
    "CFG1",
    "CFG2",
    "qam_table",
    "qam_modulate",
    "pilot_owner",
    "tdl_profile",
    "make_slot",
    "make_batch",
    "uneven_cells",
]


@dataclasses.dataclass(frozen=True)
class SlotConfig:
    """Shape and channel of one synthetic PUSCH slot (Sec. II use-case parameters)."""

    n_ant: int  # N_R receive antennas
    n_fft: int  # N, FFT size
    n_sc: int  # N_act active subcarriers (<= n_fft)
    n_symb: int  # OFDM symbols per slot
    pilot_symb: tuple  # 0-based pilot symbol indices, ascending
    n_beams: int  # N_B beams
    n_ue: int  # N_L UEs
    qam_bits: int  # bits per data symbol (2, 4, 6 or 8)
    channel: str = "flat"  # "flat" or "tdl"
    snr_db: float | None = 20.0  # None => noiseless
    tdl_rms_ns: float = 300.0
    tdl_taps: int = 8
    scs_hz: float = 30e3
    doppler_hz: float = 0.0  # > 0: every tap of every (antenna, UE) pair turns at f_D cos(theta) over the slot
    comb_aligned: bool = False  # True: every pilot symbol puts each UE's pilots on the same subcarriers

    @property
    def n_pilot(self) -> int:
        return len(self.pilot_symb)

    @property
    def data_symb(self) -> tuple:
        return tuple(s for s in range(self.n_symb) if s not in self.pilot_symb)

    @property
    def n_data(self) -> int:
        return self.n_symb - self.n_pilot

    @property
    def sigma2(self) -> float:
        return 0.0 if self.snr_db is None else 10.0 ** (-self.snr_db / 10.0)

    def replace(self, **kw) -> "SlotConfig":
        return dataclasses.replace(self, **kw)


# 16 antennas, 256-point FFT (all subcarriers used), pilot QPSK on symbol 2,
# 16 beams, 4 UEs with 16-QAM, flat i.i.d. CN(0,1) channel, 20 dB.
CFG1 = SlotConfig(n_ant=16, n_fft=256, n_sc=256, n_symb=14, pilot_symb=(2,),
                  n_beams=16, n_ue=4, qam_bits=4, channel="flat", snr_db=20.0)

# 64 antennas, 4096-point FFT with 3300 active subcarriers, pilots on symbols
# 2 and 11, 32 beams, 16 UEs with 64-QAM, 8-tap exponential-PDP channel with
# 300 ns RMS delay spread at 30 kHz subcarrier spacing.
CFG2 = SlotConfig(n_ant=64, n_fft=4096, n_sc=3300, n_symb=14, pilot_symb=(2, 11),
                  n_beams=32, n_ue=16, qam_bits=6, channel="tdl", snr_db=20.0)


def qam_table(bits: int) -> tuple[np.ndarray, np.ndarray]:
    """Gray-mapped square QAM with unit average energy (3GPP TS 38.211 Sec. 5.1).

    Returns (points[2**bits] complex128, labels[2**bits, bits] uint8) where
    point i carries bit pattern labels[i] (MSB-first, b(0) first).
    """
    if bits not in (2, 4, 6, 8):
        raise ValueError(f"unsupported QAM order: {bits} bits/symbol")
    idx = np.arange(1 << bits)
    labels = ((idx[:, None] >> (bits - 1 - np.arange(bits))[None, :]) & 1).astype(np.uint8)
    s = 1.0 - 2.0 * labels  # (1 - 2 b(i))
    half = bits // 2
    # Each rail nests (1-2b) factors: rail = s0 * (2^{h-1} - s2 * (2^{h-2} - s4 * (...)))
    def rail(first: int) -> np.ndarray:
        val = np.ones(len(idx))
        for level in range(half - 1, 0, -1):
            val = (1 << (half - level)) - s[:, first + 2 * level] * val
        return s[:, first] * val
    norm = {2: math.sqrt(2.0), 4: math.sqrt(10.0), 6: math.sqrt(42.0), 8: math.sqrt(170.0)}[bits]
    pts = (rail(0) + 1j * rail(1)) / norm
    return pts, labels


def qam_modulate(bit_array: np.ndarray, bits: int) -> np.ndarray:
    """Map bit groups [..., bits] to QAM symbols via qam_table."""
    pts, _ = qam_table(bits)
    weights = 1 << (bits - 1 - np.arange(bits))
    return pts[(bit_array.astype(np.int64) * weights).sum(-1)]


def pilot_owner(n_sc: int, j: int, n_ue: int, n_pilot: int, aligned: bool = False) -> np.ndarray:
    """UE index whose pilot sits on each subcarrier of pilot symbol j (comb with stagger, or without
    when aligned)."""
    o_j = 0 if aligned else j * (n_ue // n_pilot)
    return (np.arange(n_sc) + o_j) % n_ue


def tdl_profile(n_taps: int, rms_s: float) -> tuple[np.ndarray, np.ndarray]:
    """Exponential power-delay profile P_t ~ exp(-t), uniform tap delays, given RMS spread.

    Returns (powers summing to 1, delays in seconds).
    """
    t = np.arange(n_taps, dtype=np.float64)
    p = np.exp(-t)
    p /= p.sum()
    mean = (p * t).sum()
    rms_units = math.sqrt((p * t * t).sum() - mean * mean)
    delta = rms_s / rms_units
    return p, t * delta


def _cn(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    """Circularly-symmetric complex Gaussian samples with the given variance."""
    z = rng.standard_normal(shape + (2,))
    return (z[..., 0] + 1j * z[..., 1]) * math.sqrt(var / 2.0)


def make_slot(cfg: SlotConfig, seed: int, sigma2: float | None = None) -> dict:
    """Generate one slot.

    Returns a dict with
      x_td   complex64 [n_symb][n_ant][n_fft]   received time-domain samples
      pilots complex64 [n_pilot][n_sc]          pilot value on each pilot RE
      data   complex128 [n_data][n_ue][n_sc]    transmitted data symbols
      bits   uint8 [n_data][n_ue][n_sc][qam_bits]
      h_ant  complex128 [n_sc][n_ant][n_ue]     antenna-domain channel (at symbol 0 with Doppler;
                                                [n_symb][n_sc][n_ant][n_ue] as h_ant_t)
      grid   complex128 [n_symb][n_ant][n_sc]   noiseless received frequency grid
      sigma2 float                              noise variance per RE
    """
    rng = np.random.default_rng(seed)
    s2 = cfg.sigma2 if sigma2 is None else float(sigma2)
    if cfg.n_sc > cfg.n_fft or cfg.n_ue < 1 or cfg.n_pilot < 1:
        raise ValueError("inconsistent slot configuration")
    D, L, K, R, N = cfg.n_data, cfg.n_ue, cfg.n_sc, cfg.n_ant, cfg.n_fft

    bits = rng.integers(0, 2, size=(D, L, K, cfg.qam_bits), dtype=np.uint8)
    data = qam_modulate(bits, cfg.qam_bits)
    pbits = rng.integers(0, 2, size=(cfg.n_pilot, K, 2), dtype=np.uint8)
    pilots = qam_modulate(pbits, 2)

    if cfg.channel == "flat":
        taps = _cn(rng, (1, R, L), 1.0)
        phase = np.ones((K, 1))
    elif cfg.channel == "tdl":
        p, tau = tdl_profile(cfg.tdl_taps, cfg.tdl_rms_ns * 1e-9)
        taps = _cn(rng, (cfg.tdl_taps, R, L), 1.0) * np.sqrt(p)[:, None, None]
        kappa = np.arange(K) - K // 2
        phase = np.exp(-2j * np.pi * np.outer(kappa * cfg.scs_hz, tau))  # [K][taps]
    else:
        raise ValueError(f"unknown channel model {cfg.channel!r}")
    h_ant = np.tensordot(phase, taps, axes=(1, 0))  # [K][R][L]

    # Transmitted frequency grid per UE: [n_symb][n_ue][n_sc]
    tx = np.zeros((cfg.n_symb, L, K), dtype=np.complex128)
    for d, s in enumerate(cfg.data_symb):
        tx[s] = data[d]
    for j, s in enumerate(cfg.pilot_symb):
        owner = pilot_owner(K, j, L, cfg.n_pilot, cfg.comb_aligned)
        tx[s, owner, np.arange(K)] = pilots[j]

    # Time variation (drawn last, so slots without it keep their values): tap t
    # of pair (r, l) turns by 2 pi f_D cos(theta) per second, one symbol lasting
    # 1 / scs (no cyclic prefix)
    if cfg.doppler_hz > 0:
        theta = rng.uniform(0.0, 2.0 * np.pi, size=taps.shape)
        sym = np.arange(cfg.n_symb)[:, None, None, None] / cfg.scs_hz
        rot = np.exp(2j * np.pi * cfg.doppler_hz * np.cos(theta)[None] * sym)  # [S][taps][R][L]
        h_t = np.einsum("kt,strl->skrl", phase, taps[None] * rot, optimize=True)
    else:
        h_t = np.broadcast_to(h_ant, (cfg.n_symb,) + h_ant.shape)

    # Received noiseless grid R[s][r][k] = sum_l H_s[k][r][l] X[s][l][k]
    grid = np.einsum("skrl,slk->srk", h_t, tx, optimize=True)
    full = np.zeros((cfg.n_symb, R, N), dtype=np.complex128)
    bins = (np.arange(K) - K // 2) % N
    full[:, :, bins] = grid
    x_td = np.fft.ifft(full, axis=-1)
    if s2 > 0:
        x_td = x_td + _cn(rng, x_td.shape, s2 / N)
    return {
        "x_td": x_td.astype(np.complex64),
        "pilots": pilots.astype(np.complex64),
        "data": data,
        "bits": bits,
        "h_ant": h_ant,
        "h_ant_t": np.asarray(h_t),
        "grid": grid,
        "sigma2": s2,
    }


def make_batch(cfg: SlotConfig, seeds, sigma2: float | None = None, keep=("x_td", "pilots", "data", "bits")) -> dict:
    """Stack several slots (one seed each) along a new leading axis."""
    slots = [make_slot(cfg, int(s), sigma2) for s in seeds]
    out = {k: np.stack([sl[k] for sl in slots]) for k in keep}
    out["sigma2"] = slots[0]["sigma2"]
    return out


def uneven_cells(n_cells: int, seed: int = 4000) -> list[dict]:
    """Seeded draw of uneven cells: FFT size in {1024, 2048, 4096} with
    N * 3300 / 4096 active subcarriers, 16/32/64 antennas, beams = antennas / 2,
    4..16 UEs, pilots on symbols 2 and 11, one slot each, sigma^2 = 0.01."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_cells):
        n_fft = int(rng.choice([1024, 2048, 4096]))
        n_ant = int(rng.choice([16, 32, 64]))
        n_beams = n_ant // 2
        n_ue = int(rng.integers(4, min(16, n_beams) + 1))
        out.append(dict(n_ant=n_ant, n_fft=n_fft, n_sc=n_fft * 3300 // 4096, n_symb=14, n_beams=n_beams, n_ue=n_ue,
                        pilot_symb=(2, 11), sigma2=0.01, n_slot=1))
    return out
