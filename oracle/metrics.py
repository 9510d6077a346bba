"""Error and quality metrics used to score results against the oracle.

TEST INFRASTRUCTURE ONLY (see the header of pusch_oracle).

Each function is pinned in tests/test_oracle.py by hand-worked values that the
mathematics fixes (not by re-typing its formula), and planted mistakes in a
copy of this module (squared ratio, wrong normalisation, 20 log10, reversed
margin, ...) are checked to fail those pins.
"""
from __future__ import annotations

import numpy as np


def nrmse(a, ref) -> float:
    """Normalised RMS error ||a - ref||_2 / ||ref||_2 over the whole tensor."""
    a = np.asarray(a, np.complex128)
    ref = np.asarray(ref, np.complex128)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((a - ref).ravel()) / (den if den > 0 else 1.0))


def max_rel_err(a, ref) -> float:
    """Largest element error relative to the RMS magnitude of the reference."""
    a = np.asarray(a, np.complex128)
    ref = np.asarray(ref, np.complex128)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2)) if ref.size else 1.0
    return float(np.max(np.abs(a - ref)) / (rms if rms > 0 else 1.0)) if ref.size else 0.0


def worst_slice_err(a, ref, axis: int) -> float:
    """Largest RMS error over one index of `axis` (every other axis pooled),
    relative to the RMS magnitude of the whole reference.

    With axis = the subcarrier axis this is the worst subcarrier's error in
    units of the tensor's RMS: a wrong block of subcarriers shows up here even
    when it is too small a share of the tensor to move nrmse."""
    a = np.asarray(a, np.complex128)
    ref = np.asarray(ref, np.complex128)
    if ref.size == 0:
        return 0.0
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    other = tuple(i for i in range(ref.ndim) if i != axis % ref.ndim)
    per = np.sqrt(np.mean(np.abs(a - ref) ** 2, axis=other))
    return float(np.max(per) / (rms if rms > 0 else 1.0))


def evm_db(x_hat, x) -> float:
    """Error vector magnitude in dB over all data REs and UEs: 10 log10 of the
    error power over the reference power (a power ratio, hence 10, not 20)."""
    x_hat = np.asarray(x_hat, np.complex128)
    x = np.asarray(x, np.complex128)
    return float(10.0 * np.log10(np.sum(np.abs(x_hat - x) ** 2) / np.sum(np.abs(x) ** 2)))


def hard_decide(x_hat, points, labels) -> tuple[np.ndarray, np.ndarray]:
    """Nearest-constellation-point decision (lowest index wins a tie).

    Returns (symbol index array, bits [..., bits_per_symbol])."""
    x_hat = np.asarray(x_hat, np.complex128)
    d = np.abs(x_hat[..., None] - np.asarray(points)[None, :]) ** 2
    idx = np.argmin(d, axis=-1)
    return idx, np.asarray(labels)[idx]


def decision_margin(x_hat, points) -> np.ndarray:
    """Distance gap between the nearest and second-nearest constellation point
    (how far a soft value sits from a decision boundary, in squared-distance units)."""
    x_hat = np.asarray(x_hat, np.complex128)
    d = np.sort(np.abs(x_hat[..., None] - np.asarray(points)[None, :]) ** 2, axis=-1)
    return d[..., 1] - d[..., 0]


def xhat_errors(a, ref, sc_axis: int = -2) -> dict:
    """The three figures every detected-symbol parity check bounds:
    whole-tensor NRMSE, the largest element error and the worst subcarrier's
    RMS error (both relative to the reference RMS).  Detected symbols are laid
    out [..., n_sc, n_ue], so the subcarrier axis defaults to -2."""
    return {"nrmse": nrmse(a, ref), "max_rel": max_rel_err(a, ref), "worst_sc": worst_slice_err(a, ref, sc_axis)}
