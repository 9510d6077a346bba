"""FP64 CPU oracle of the learned LS-channel-estimate denoiser and of the pilot
residual that decides when the chain falls back to plain LS.

TEST INFRASTRUCTURE ONLY (see the header of pusch_oracle): only the test
suite, the package entry file's smoke check and the CPU baseline of the
benchmark may import this module; the HIP product path never calls it.

What is computed.  The paper's channel estimator is least squares on the
pilot symbols (Sec. II, CHE; Table 1, row "CHE").  The denoiser refines that
estimate: for every (UE, beam) pair the LS estimate over the subcarrier x
symbol grid (real and imaginary parts as two channels) passes four 3x3
convolution layers of 32 channels, 2 -> 32 -> 32 -> 32 -> 2, with ReLU after
the first three, and the network's output is added to the LS estimate
(a residual correction).  Convolutions are cross-correlations over (symbol,
subcarrier) with zero padding ("same" size).

Parameters live in one flat FP32 vector, layer by layer: W_l[c_out][dy][dx][c_in]
(input channel fastest), then b_l[c_out].

With bf16=True the oracle rounds, to bfloat16 (round to nearest, ties to
even), exactly the values the GPU kernels hold in bfloat16: the weights, the
network input, the three hidden activations, and the output gradients fed to
the transposed convolutions; everything else stays FP64.  The GPU path then
differs from it only by FP32 accumulation order.

Readings (where the paper gives no denoiser at all):
  R19 LS grid over all symbols: each symbol's estimate is the time
      interpolation of R18 between the per-pilot-symbol LS estimates (held
      outside), so with one pilot symbol it is the same on every symbol.
  R20 fallback: the "post-MMSE pilot residual" of an estimator is measured on
      held-out pilots.  Each UE's pilot positions on each pilot symbol are
      split by their order along k into an even and an odd half; the
      estimator sees one half, and at every pilot RE of the other half the
      MMSE-equalised received vector (Eq. 2 with that estimate) is compared
      with the known transmitted vector (the UE's pilot, zero for the other
      UEs).  Both halves take a turn; the residual is the summed squared
      error.  The chain keeps the denoised estimate unless its residual
      exceeds the LS one.  (On the full comb the LS estimate passes through
      every pilot RE, so a residual on seen pilots would always favour LS.)
"""
from __future__ import annotations

import numpy as np

from oracle import pusch_oracle as O

LAYERS = ((2, 32, True), (32, 32, True), (32, 32, True), (32, 2, False))  # (c_in, c_out, relu)


def param_shapes() -> list[tuple[tuple, tuple]]:
    return [((co, 3, 3, ci), (co,)) for ci, co, _ in LAYERS]


def n_params() -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def unpack(params) -> list[tuple[np.ndarray, np.ndarray]]:
    """Flat parameter vector -> [(W [co][3][3][ci], b [co]) per layer]."""
    p = np.asarray(params, np.float64).ravel()
    if p.size != n_params():
        raise ValueError(f"expected {n_params()} parameters, got {p.size}")
    out, o = [], 0
    for ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((p[o:o + nw].reshape(ws), p[o + nw:o + nw + nb].reshape(bs)))
        o += nw + nb
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([np.ravel(W), np.ravel(b)]) for W, b in layers])


def to_bf16(x) -> np.ndarray:
    """Round to bfloat16 (8 significant bits), nearest, ties to even; returned as float64.

    FP32 bit pattern u; the kept part is u >> 16, rounded by adding 0x7FFF plus the
    kept part's lowest bit before truncating (non-finite inputs are not used here)."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, W, b=None) -> np.ndarray:
    """'Same' 3x3 cross-correlation with zero padding.

    x: [S, K, c_in]; W: [c_out, 3, 3, c_in]; b: [c_out] or None.
    out[s, k, o] = b[o] + sum_{dy, dx, i} W[o, dy, dx, i] x[s + dy - 1, k + dx - 1, i]."""
    x = np.asarray(x, np.float64)
    S, K, _ = x.shape
    xp = np.zeros((S + 2, K + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    out = np.zeros((S, K, W.shape[0]))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("ski,oi->sko", xp[dy:dy + S, dx:dx + K], W[:, dy, dx, :])
    if b is not None:
        out += b
    return out


def conv3x3_transposed(g, W) -> np.ndarray:
    """Gradient of conv3x3 with respect to its input: dx[s, k, i] =
    sum_{o, dy, dx} W[o, dy, dx, i] g[s - dy + 1, k - dx + 1, o] (zero outside).

    g: [S, K, c_out]; W: [c_out, 3, 3, c_in].  Returns [S, K, c_in]."""
    g = np.asarray(g, np.float64)
    S, K, _ = g.shape
    gp = np.zeros((S + 2, K + 2, g.shape[2]))
    gp[1:-1, 1:-1] = g
    out = np.zeros((S, K, W.shape[3]))
    for dy in range(3):
        for dx in range(3):
            # x[s, k] reaches out[s', k'] through (dy, dx) when s' = s - dy + 1
            out += np.einsum("sko,oi->ski", gp[2 - dy:2 - dy + S, 2 - dx:2 - dx + K], W[:, dy, dx, :])
    return out


def conv3x3_weight_grad(g, x) -> tuple[np.ndarray, np.ndarray]:
    """Gradients of conv3x3 with respect to W and b: dW[o, dy, dx, i] =
    sum_{s, k} g[s, k, o] x[s + dy - 1, k + dx - 1, i]; db[o] = sum g[s, k, o]."""
    g = np.asarray(g, np.float64)
    x = np.asarray(x, np.float64)
    S, K, _ = x.shape
    xp = np.zeros((S + 2, K + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    dW = np.zeros((g.shape[2], 3, 3, x.shape[2]))
    for dy in range(3):
        for dx in range(3):
            dW[:, dy, dx, :] = np.einsum("sko,ski->oi", g, xp[dy:dy + S, dx:dx + K])
    return dW, g.sum(axis=(0, 1))


def forward(grid, params, bf16: bool = False):
    """Denoised estimate of one LS grid [S, K] (complex): grid + net(grid).

    Returns (out [S, K] complex128, cache for backward)."""
    grid = np.asarray(grid, np.complex128)
    rnd = to_bf16 if bf16 else (lambda v: np.asarray(v, np.float64))
    layers = unpack(params)
    a = rnd(np.stack([grid.real, grid.imag], axis=-1))
    acts = [a]  # the input of every layer, as the layer reads it
    for n, ((W, b), (_, _, relu)) in enumerate(zip(layers, LAYERS)):
        z = conv3x3(a, rnd(W), b)
        if relu:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
        else:
            a = z
    out = grid + (a[..., 0] + 1j * a[..., 1])
    return out, {"acts": acts, "bf16": bf16, "layers": layers}


def backward(cache, dout) -> np.ndarray:
    """Gradient of a loss with respect to the flat parameters, given dL/d(out)
    as a complex grid whose real and imaginary parts are the derivatives with
    respect to the output's real and imaginary parts."""
    bf16 = cache["bf16"]
    rnd = to_bf16 if bf16 else (lambda v: np.asarray(v, np.float64))
    acts, layers = cache["acts"], cache["layers"]
    dout = np.asarray(dout, np.complex128)
    g = np.stack([dout.real, dout.imag], axis=-1)  # dL/dz of the last layer
    grads = [None] * len(layers)
    for n in range(len(layers) - 1, -1, -1):
        W, _ = layers[n]
        grads[n] = conv3x3_weight_grad(g, acts[n])
        if n == 0:
            break
        da = conv3x3_transposed(rnd(g), rnd(W))
        g = da * (acts[n] > 0)  # ReLU of layer n - 1: its output acts[n]
    return pack(grads)


def mse_loss(out, target) -> tuple[float, np.ndarray]:
    """Mean over all complex entries of |out - target|^2, and its gradient as a
    complex grid (d/d re + i d/d im): 2 (out - target) / N."""
    out = np.asarray(out, np.complex128)
    target = np.asarray(target, np.complex128)
    e = out - target
    n = e.size
    return float(np.sum(e.real ** 2 + e.imag ** 2) / n), 2.0 * e / n


# ----------------------------------------------------------------------------- LS grid and fallback

def _fold_positions(ks: np.ndarray, fold: int) -> np.ndarray:
    """A UE's pilot subcarriers on one pilot symbol (ascending): all (fold 0), the
    even-indexed half (fold 1) or the odd-indexed half (fold 2)."""
    return ks if fold == 0 else ks[fold - 1::2]


def ls_symbol_estimate(Yp_j, p_j, n_ue: int, j: int, n_pilot: int, fold: int = 0) -> np.ndarray:
    """LS estimate from pilot symbol j alone (as pusch_oracle.ls_channel_estimate
    with use=[j]), from the fold's positions only.  Yp_j: [N_B, K]; p_j: [K].
    Returns [K, N_B, N_L]."""
    n_beams, K = Yp_j.shape
    H = np.zeros((K, n_beams, n_ue), complex)
    grid = np.arange(K, dtype=np.float64)
    owner = O.pilot_owner(K, j, n_ue, n_pilot)
    for l in range(n_ue):
        ks = _fold_positions(np.nonzero(owner == l)[0], fold)
        p = p_j[ks]
        val = Yp_j[:, ks] * (np.conj(p) / np.abs(p) ** 2)
        for b in range(n_beams):
            H[:, b, l] = np.interp(grid, ks, val[b].real) + 1j * np.interp(grid, ks, val[b].imag)
    return H


def ls_grid(Yp, pilots, n_ue: int, pilot_symb, n_symb: int, fold: int = 0) -> np.ndarray:
    """LS estimate on every symbol (reading R19): per pilot symbol from its own
    positions (of the fold), interpolated linearly in time between the pilot
    symbols around each symbol and held outside them.

    Yp: [N_p, N_B, K]; pilots: [N_p, K].  Returns [S, K, N_B, N_L]."""
    Yp = np.asarray(Yp, np.complex128)
    pilots = np.asarray(pilots, np.complex128)
    n_pilot = Yp.shape[0]
    per = [ls_symbol_estimate(Yp[j], pilots[j], n_ue, j, n_pilot, fold) for j in range(n_pilot)]
    ps = list(pilot_symb)
    out = []
    for s in range(n_symb):
        if s <= ps[0]:
            out.append(per[0])
        elif s >= ps[-1]:
            out.append(per[-1])
        else:
            b = next(j for j, q in enumerate(ps) if q > s)
            a = b - 1
            out.append(((ps[b] - s) * per[a] + (s - ps[a]) * per[b]) / (ps[b] - ps[a]))
    return np.stack(out)


def denoise_estimate(H_grid, params, bf16: bool = False) -> np.ndarray:
    """The network on every (beam, UE) pair of an estimate [S, K, N_B, N_L]."""
    S, K, NB, NL = H_grid.shape
    out = np.zeros_like(H_grid)
    for b in range(NB):
        for l in range(NL):
            out[:, :, b, l] = forward(H_grid[:, :, b, l], params, bf16)[0]
    return out


def pilot_holdout_residual(Yp, pilots, n_ue: int, pilot_symb, n_symb: int, sigma2: float, estimator) -> float:
    """Post-MMSE pilot residual of an estimator (reading R20).

    estimator(fold) -> [S, K, N_B, N_L] estimate from that fold's pilots.  For
    fold 1 the held-out REs are fold 2's and vice versa.  At each held-out
    pilot RE (j, k) of UE l the received vector is equalised with Eq. 2 using
    the estimate of symbol pilot_symb[j] at k, and |x_hat - p e_l|^2 is summed."""
    Yp = np.asarray(Yp, np.complex128)
    pilots = np.asarray(pilots, np.complex128)
    n_pilot, _, K = Yp.shape
    total = 0.0
    for fold, held in ((1, 2), (2, 1)):
        H = estimator(fold)
        for j in range(n_pilot):
            owner = O.pilot_owner(K, j, n_ue, n_pilot)
            ks = np.concatenate([_fold_positions(np.nonzero(owner == l)[0], held) for l in range(n_ue)])
            ks.sort()
            Hk = H[pilot_symb[j]][ks]  # [n, N_B, N_L]
            x_hat, _ = O.mmse_detect(Hk, Yp[j][:, ks].T[None], sigma2)
            x = np.zeros((len(ks), n_ue), complex)
            x[np.arange(len(ks)), owner[ks]] = pilots[j, ks]
            total += float(np.sum(np.abs(x_hat[0] - x) ** 2))
    return total
