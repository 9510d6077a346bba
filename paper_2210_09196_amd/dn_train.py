"""Training of the LS-estimate denoiser on the GPU with the library's kernels.

Every step draws a batch of slots of the small workload's shape (16 receive
antennas, 256 subcarriers, 14 symbols, pilot symbol 2, the 16 x 16 DFT
beamformer, 4 UEs on a comb) from the project's channel model, here drawn on
the device: an 8-tap exponential power-delay profile whose RMS delay spread is
uniform in 30..1000 ns, every tap of every (antenna, UE) pair turning at
f_D cos(theta) with f_D uniform in 0..300 Hz (one symbol lasting 1/SCS), and
an SNR uniform in 0..30 dB.  The device draws only what the transmitter and
the channel produce -- antenna-domain channels, QPSK pilots, the noise after
the unitary beamformer (white, of the same variance) -- and the library does
every receiver step: the beamforming of the channel (pusch_beamform), the LS
grid (pusch_dn_ls_grid), the network (pusch_dn_forward), the mean squared
error against the true beam-domain channel on the pilot symbols, carried over
the slot as the LS grid is (pusch_dn_loss), the gradients
(pusch_dn_backward) and the Adam step (pusch_dn_adam).

Usage: python -m paper_2210_09196_amd.dn_train --slots 200000 --out weights.npy
"""
from __future__ import annotations

import argparse
import math
import sys
import time

import numpy as np
import torch

from . import pusch

# the small workload's geometry
N_ANT, N_SC, N_SYMB, PILOT_SYMB, N_BEAMS, N_UE = 16, 256, 14, (2,), 16, 4
SCS_HZ = 30e3
TDL_TAPS = 8


def init_params(gen: torch.Generator, device) -> torch.Tensor:
    """He-normal weights (std sqrt(2 / (9 c_in))), zero biases, the last layer scaled by 0.1 so the
    untrained network starts close to the plain LS estimate.  Layout as the library's."""
    parts = []
    layers = ((2, 32), (32, 32), (32, 32), (32, 2))
    for n, (ci, co) in enumerate(layers):
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if n == 3 else 1.0)
        parts.append(torch.randn(co * 9 * ci, generator=gen, device=device) * std)
        parts.append(torch.zeros(co, device=device))
    p = torch.cat(parts).contiguous()
    assert p.numel() == pusch.DN_PARAMS
    return p


def time_weights(n_symb: int, pilot_symb) -> list[list[float]]:
    """Weight of each pilot symbol in symbol s's estimate: held before the first and after the
    last pilot symbol, linear in time between the two around s (as the LS grid)."""
    ps = list(pilot_symb)
    w = []
    for s in range(n_symb):
        row = [0.0] * len(ps)
        if s <= ps[0]:
            row[0] = 1.0
        elif s >= ps[-1]:
            row[-1] = 1.0
        else:
            b = next(j for j, q in enumerate(ps) if q > s)
            row[b - 1] = (ps[b] - s) / (ps[b] - ps[b - 1])
            row[b] = (s - ps[b - 1]) / (ps[b] - ps[b - 1])
        w.append(row)
    return w


def _cis(a: torch.Tensor) -> torch.Tensor:
    """exp(i a), complex64."""
    return torch.complex(torch.cos(a), torch.sin(a))


def _cn(gen, shape, device) -> torch.Tensor:
    """CN(0, 1) samples, complex64."""
    z = torch.randn(*shape, 2, generator=gen, device=device) * math.sqrt(0.5)
    return torch.view_as_complex(z).contiguous()


def draw_batch(gen: torch.Generator, n_slot: int, device, rms_ns=(30.0, 1000.0), doppler_hz=(0.0, 300.0),
               snr_db=(0.0, 30.0)):
    """One batch of training pairs: (LS grid, true beam-domain channel), both complex64
    [n_slot * N_UE * N_BEAMS, N_SYMB, N_SC] in the library's grid order (slot, UE, beam), and the
    noise variance of each grid's slot ([n_slot * N_UE * N_BEAMS] float32)."""
    G, S, K, R, L, T = n_slot, N_SYMB, N_SC, N_ANT, N_UE, TDL_TAPS
    u = lambda lo, hi: lo + (hi - lo) * torch.rand(G, generator=gen, device=device)
    rms = u(*rms_ns) * 1e-9
    fd = u(*doppler_hz)
    s2 = 10.0 ** (-u(*snr_db) / 10.0)
    # exponential power-delay profile, uniform tap spacing giving the drawn RMS delay spread
    t = torch.arange(T, dtype=torch.float32, device=device)
    pw = torch.exp(-t)
    pw = pw / pw.sum()
    mean = (pw * t).sum()
    rms_units = torch.sqrt((pw * t * t).sum() - mean * mean)
    tau = t[None, :] * (rms / rms_units)[:, None]  # [G][T] seconds
    taps = _cn(gen, (G, T, L, R), device) * torch.sqrt(pw)[None, :, None, None]
    theta = 2 * math.pi * torch.rand(G, T, L, R, generator=gen, device=device)
    sym_t = torch.arange(S, dtype=torch.float32, device=device) / SCS_HZ
    rot = _cis(2 * math.pi * fd[:, None, None, None, None] * torch.cos(theta)[:, None] * sym_t[None, :, None, None, None])
    kappa = torch.arange(K, dtype=torch.float32, device=device) - K // 2
    phase = _cis(-2 * math.pi * SCS_HZ * kappa[None, :, None] * tau[:, None, :])
    # H_ant[g][s][l][r][k] = sum_t taps * rot * phase
    h = torch.einsum("gkt,gstlr->gslrk", phase, taps[:, None] * rot).contiguous()
    # beam-domain channel through the library's beamforming: [g s l][k][b]
    hb = pusch.beamform(h.view(G * S * L, R, K), N_BEAMS)
    hb = hb.view(G, S, L, K, N_BEAMS)
    # target: the true channel on the pilot symbols at every subcarrier, carried to the other
    # symbols as the LS grid carries its estimate (held outside the pilot symbols, linear in time
    # between them).  The network removes the noise and the frequency-interpolation error of the
    # estimate; the channel's change between pilot symbols is invisible to any estimate from them.
    wt = torch.tensor(time_weights(S, PILOT_SYMB), dtype=torch.float32, device=device).to(torch.complex64)
    target = torch.einsum("sj,gjlkb->glbsk", wt, hb[:, list(PILOT_SYMB)]).contiguous().view(G * L * N_BEAMS, S, K)
    # received pilot symbol: each subcarrier carries its comb owner's QPSK pilot, plus white noise
    ps = PILOT_SYMB[0]
    owner = torch.arange(K, device=device) % L
    pil = _cis((math.pi / 2) * torch.randint(0, 4, (G, 1, K), generator=gen, device=device).float()
               + math.pi / 4).contiguous()
    hp = hb[:, ps, owner, torch.arange(K, device=device), :]  # [G][K][B]
    noise = _cn(gen, (G, K, N_BEAMS), device) * torch.sqrt(s2)[:, None, None]
    Yp = (hp * pil[:, 0, :, None] + noise).view(G, 1, K, N_BEAMS).contiguous()
    grid = pusch.dn_ls_grid(Yp, pil, N_UE, S, PILOT_SYMB)
    return grid.view(G * L * N_BEAMS, S, K), target, s2.repeat_interleave(L * N_BEAMS).contiguous()


def train(n_slots: int, batch_slots: int = 16, lr: float = 2e-3, seed: int = 1, device="cuda", log_every: int = 100,
          params: torch.Tensor | None = None):
    """Adam with a cosine learning-rate decay over n_slots / batch_slots steps; returns
    (params, history of (step, loss, LS loss)).  The network is trained in units of the noise
    standard deviation: its input is the LS grid divided by sigma of the grid's slot and its target
    the true channel divided by the same sigma (the chain runs it so: pusch_slot_denoised divides by
    sqrt(sigma2) and scales the correction back).  The network then sees unit noise at every SNR,
    and the squared error counts in units of the noise -- what the detector loses to an estimation
    error grows with its size relative to the noise, so a grid at 30 dB counts as much as one at
    0 dB."""
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    p = init_params(gen, device) if params is None else params.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    n_grid = batch_slots * N_UE * N_BEAMS
    net = pusch.Denoiser(N_SYMB, N_SC, n_grid, device=device)
    out = torch.empty(n_grid, N_SYMB, N_SC, dtype=torch.complex64, device=device)
    dout = torch.empty_like(out)
    grads = torch.empty_like(p)
    steps = max(1, n_slots // batch_slots)
    hist = []
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        grid, target, s2 = draw_batch(gen, batch_slots, device)
        inv = torch.rsqrt(s2)[:, None, None]
        grid = (grid * inv).contiguous()
        target = (target * inv).contiguous()
        net.forward(p, grid, out)
        loss, _ = net.loss(out, target, dout)
        net.backward(p, grid, dout, grads)
        rate = 1e-5 + 0.5 * (lr - 1e-5) * (1 + math.cos(math.pi * (step - 1) / steps))
        pusch.dn_adam(p, grads, m, v, step, rate)
        if step % log_every == 0 or step == steps:
            ls = float(((grid - target).abs() ** 2).mean())
            lv = float(loss.item())
            hist.append((step, lv, ls))
            print(f"[dn_train] step {step}/{steps} loss {lv:.5f} (LS {ls:.5f}, ratio {lv / ls:.3f}), "
                  f"{time.perf_counter() - t0:.1f} s", flush=True)
    return p, hist


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--slots", type=int, default=200000, help="generated slots in all")
    ap.add_argument("--batch", type=int, default=16, help="slots per step (64 grids each)")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", required=True, help="where to save the trained parameters (.npy, float32)")
    args = ap.parse_args(argv)
    p, hist = train(args.slots, args.batch, args.lr, args.seed)
    np.save(args.out, p.cpu().numpy().astype(np.float32), allow_pickle=False)
    print(f"[dn_train] saved {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
