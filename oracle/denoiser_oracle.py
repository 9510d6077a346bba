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
  R20 fallback: the "post-MMSE residual" of an estimate is measured on the
      data REs: each data symbol is equalised with Eq. 2 using the estimate,
      and |y - H_hat x_hat|^2 is summed over the slot's data REs and beams.
      Neither estimate has seen those REs, so the sum grows with the
      estimation error.  The chain keeps the denoised estimate unless its
      residual exceeds the LS one.  (The LS estimate passes through every
      pilot RE of its comb, so a residual on the pilot REs would always favour
      it; held-out pilots of a regular comb sit where linear interpolation is
      at its best, at the midpoints between the seen ones.)
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


def forward(grid, params, bf16: bool = False, sigma: float = 1.0):
    """Denoised estimate of one LS grid [S, K] (complex): grid + sigma net(grid / sigma),
    the network run in units of sigma (sigma = 1: the plain network).

    Returns (out [S, K] complex128, cache for backward, valid for sigma = 1)."""
    grid = np.asarray(grid, np.complex128)
    rnd = to_bf16 if bf16 else (lambda v: np.asarray(v, np.float64))
    layers = unpack(params)
    x = grid / sigma
    a = rnd(np.stack([x.real, x.imag], axis=-1))
    acts = [a]  # the input of every layer, as the layer reads it
    for n, ((W, b), (_, _, relu)) in enumerate(zip(layers, LAYERS)):
        z = conv3x3(a, rnd(W), b)
        if relu:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
        else:
            a = z
    out = grid + sigma * (a[..., 0] + 1j * a[..., 1])
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


def mse_loss(out, target, weights=None) -> tuple[float, np.ndarray]:
    """Mean over all complex entries of w_g |out - target|^2 (grids g along the
    first axis, w_g = 1 without weights), and its gradient as a complex grid
    (d/d re + i d/d im): 2 w_g (out - target) / N."""
    out = np.asarray(out, np.complex128)
    target = np.asarray(target, np.complex128)
    e = out - target
    n = e.size
    w = np.ones(e.shape[0]) if weights is None else np.asarray(weights, np.float64)
    w = w.reshape((-1,) + (1,) * (e.ndim - 1))
    return float(np.sum(w * (e.real ** 2 + e.imag ** 2)) / n), 2.0 * w * e / n


# ----------------------------------------------------------------------------- LS grid and fallback

def ls_symbol_estimate(Yp_j, p_j, n_ue: int, j: int, n_pilot: int) -> np.ndarray:
    """LS estimate from pilot symbol j alone (as pusch_oracle.ls_channel_estimate
    with use=[j]).  Yp_j: [N_B, K]; p_j: [K].  Returns [K, N_B, N_L]."""
    n_beams, K = Yp_j.shape
    H = np.zeros((K, n_beams, n_ue), complex)
    grid = np.arange(K, dtype=np.float64)
    owner = O.pilot_owner(K, j, n_ue, n_pilot)
    for l in range(n_ue):
        ks = np.nonzero(owner == l)[0]
        p = p_j[ks]
        val = Yp_j[:, ks] * (np.conj(p) / np.abs(p) ** 2)
        for b in range(n_beams):
            H[:, b, l] = np.interp(grid, ks, val[b].real) + 1j * np.interp(grid, ks, val[b].imag)
    return H


def ls_grid(Yp, pilots, n_ue: int, pilot_symb, n_symb: int) -> np.ndarray:
    """LS estimate on every symbol (reading R19): per pilot symbol from its own
    comb positions, interpolated linearly in time between the pilot symbols
    around each symbol and held outside them.

    Yp: [N_p, N_B, K]; pilots: [N_p, K].  Returns [S, K, N_B, N_L]."""
    Yp = np.asarray(Yp, np.complex128)
    pilots = np.asarray(pilots, np.complex128)
    n_pilot = Yp.shape[0]
    per = [ls_symbol_estimate(Yp[j], pilots[j], n_ue, j, n_pilot) for j in range(n_pilot)]
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


def denoise_estimate(H_grid, params, bf16: bool = False, sigma: float = 1.0) -> np.ndarray:
    """The network (in units of sigma) on every (beam, UE) pair of an estimate [S, K, N_B, N_L]."""
    S, K, NB, NL = H_grid.shape
    out = np.zeros_like(H_grid)
    for b in range(NB):
        for l in range(NL):
            out[:, :, b, l] = forward(H_grid[:, :, b, l], params, bf16, sigma)[0]
    return out


def detect_and_residual(Y, H_grid, pilot_symb, sigma2: float):
    """Eq. 2 on every data symbol with the estimate of that symbol, and the
    post-MMSE residual of reading R20: sum over data REs and beams of
    |y - H_hat x_hat|^2.

    Y: [S, N_B, K] beam-domain grids; H_grid: [S, K, N_B, N_L].
    Returns (x_hat [D, K, N_L], ok [D, K], residual)."""
    Y = np.asarray(Y, np.complex128)
    S, _, K = Y.shape
    n_ue = H_grid.shape[3]
    data = [s for s in range(S) if s not in list(pilot_symb)]
    x_hat = np.zeros((len(data), K, n_ue), complex)
    ok = np.zeros((len(data), K), bool)
    res = 0.0
    for d, s in enumerate(data):
        xs, ok[d] = O.mmse_detect(H_grid[s], Y[s].T[None], sigma2)
        x_hat[d] = xs[0]
        r = Y[s].T - np.einsum("kbl,kl->kb", H_grid[s], xs[0])
        res += float(np.sum(r.real ** 2 + r.imag ** 2))
    return x_hat, ok, res


def adam_step(p, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma and Ba, "Adam: a method for stochastic optimization",
    Algorithm 1): moments m, v of the gradient, bias-corrected by 1 - beta^step.
    Returns (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def receive_slot_denoised(x_td, pilots, pilot_symb, n_ue: int, n_sc: int, sigma2: float, params, n_beams: int,
                          W=None, bf16: bool = True) -> dict:
    """The chain with the denoised estimate and the LS fallback (reading R20):
    OFDM demodulation and beamforming as pusch_oracle.receive_slot; the LS grid
    and the network on it, in units of sqrt(sigma2); Eq. 2 for every data symbol with each estimate of
    that symbol; the denoised result unless its post-MMSE residual exceeds the
    LS one.

    Returns {"x_hat" [D, K, N_L], "used_dn" bool, "res_ls", "res_dn", "ok" [D, K]}."""
    x_td = np.asarray(x_td, np.complex128)
    n_symb, n_ant, _ = x_td.shape
    W = O.dft_beamformer(n_beams, n_ant) if W is None else np.asarray(W, np.complex128)
    Y = O.beamform(W, O.ofdm_demodulate(x_td, n_sc))  # [S, N_B, K]
    ps = list(pilot_symb)
    G = ls_grid(Y[ps], pilots, n_ue, ps, n_symb)
    # the network in units of the LS values' noise standard deviation (unit-power pilots, unitary beams)
    Dn = denoise_estimate(G, params, bf16, float(np.sqrt(sigma2)))
    x_ls, ok_ls, res_ls = detect_and_residual(Y, G, ps, sigma2)
    x_dn, ok_dn, res_dn = detect_and_residual(Y, Dn, ps, sigma2)
    use = res_dn <= res_ls
    return {"x_hat": x_dn if use else x_ls, "used_dn": bool(use), "res_ls": res_ls, "res_dn": res_dn,
            "ok": ok_dn if use else ok_ls}
