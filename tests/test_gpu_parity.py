"""GPU parity: every C-ABI entry point against the FP64 oracle.

Tolerances (FP32 path): FFT and intermediate beam-domain / channel grids
NRMSE <= 1e-5 and every element within 1e-5 of the reference RMS; detected
symbols NRMSE <= 1e-4; hard decisions identical wherever the oracle's soft
value is not within rounding distance of a decision boundary.
"""
import numpy as np
import pytest
import torch

from oracle import metrics as M
from checks import assert_xhat
from oracle import pusch_oracle as O
from paper_2210_09196_amd import pusch, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL_GRID = 1e-5  # FFT / beamforming / LS grids
TOL_X = 1e-4  # detected symbols


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_grid(got, ref, tol=TOL_GRID):
    e, m = M.nrmse(got, ref), M.max_rel_err(got, ref)
    assert e <= tol and m <= 10 * tol, f"nrmse {e:.3e} max-rel {m:.3e}"


# ----------------------------------------------------------------------------- OFDM demodulation (FFT)

ACTIVE = {64: 63, 256: 256, 1024: 825, 2048: 1650, 4096: 3300}


@pytest.mark.parametrize("n_fft", [64, 256, 1024, 2048, 4096])
@pytest.mark.parametrize("mode", ["natural", "active", "dc_only"])
def test_fft(n_fft, mode):
    rng = np.random.default_rng(n_fft)
    batch = 37  # not a multiple of the transforms per workgroup for any size
    x = crandn(rng, batch, n_fft)
    n_sc = {"natural": 0, "active": ACTIVE[n_fft], "dc_only": 1}[mode]
    X = host(pusch.fft(dev(x), n_sc))
    ref = O.ofdm_demodulate(x, None if n_sc == 0 else n_sc)
    assert_grid(X, ref)


@pytest.mark.parametrize("n_fft,n_sc", [(4096, 0), (256, 256)])
def test_fft_in_place(n_fft, n_sc):
    rng = np.random.default_rng(5)
    x = crandn(rng, 9, n_fft)
    t = dev(x)
    pusch.fft(t, n_sc, out=t)
    assert_grid(host(t), O.ofdm_demodulate(x, None if n_sc == 0 else n_sc))


def test_fft_special_inputs():
    n = 4096
    x = np.zeros((3, n), np.complex64)
    x[0, 0] = 1  # impulse -> all ones
    x[1] = np.exp(2j * np.pi * 17 * np.arange(n) / n)  # tone -> N at bin 17
    X = host(pusch.fft(dev(x)))
    assert np.max(np.abs(X[0] - 1)) < 1e-6
    assert abs(X[1, 17] - n) < 1e-2 and np.max(np.abs(np.delete(X[1], 17))) < 1e-2
    assert np.all(X[2] == 0)


def test_fft_full_size_sampled():
    # the slot batch of the throughput workload: 16 slots x 14 symbols x 64 antennas
    g = torch.Generator(device=DEV)
    g.manual_seed(2024)
    batch, n = 16 * 14 * 64, 4096
    x = torch.randn(batch, n, 2, generator=g, device=DEV)
    x = torch.view_as_complex(x).contiguous()
    X = pusch.fft(x, 3300)
    idx = np.random.default_rng(0).choice(batch, 48, replace=False)
    idx = np.concatenate([idx, [0, batch - 1]])
    xs = host(x[torch.as_tensor(idx, device=DEV)])
    assert_grid(host(X[torch.as_tensor(idx, device=DEV)]), O.ofdm_demodulate(xs, 3300))


# ----------------------------------------------------------------------------- beamforming

@pytest.mark.parametrize("nb,na,n_re,ld_x,batch,builtin", [
    (16, 16, 256, 256, 14, True),  # 16x16 DFT beamformer, 256 subcarriers
    (32, 64, 3300, 3300, 3, True),  # 64x32 DFT beamformer, 3300 subcarriers
    (32, 64, 3300, 3300, 2, False),
    (5, 7, 33, 40, 3, False),  # ragged everything, padded rows
    (64, 64, 100, 100, 2, False),
    (48, 20, 17, 17, 1, False),
    (1, 1, 1, 1, 1, False),
    # more than 64 antennas: the chunked kernel, W in LDS (first three) or read
    # from global memory (last two); 16-byte or 8-byte (odd pitch) X loads
    (16, 65, 300, 300, 2, False),
    (32, 128, 3300, 3300, 2, True),
    (64, 100, 77, 77, 3, False),
    (64, 200, 129, 131, 2, False),
    (32, 1024, 40, 40, 1, False),
])
def test_beamform(nb, na, n_re, ld_x, batch, builtin):
    rng = np.random.default_rng(nb * 1000 + na)
    X = crandn(rng, batch, na, ld_x)
    W = O.dft_beamformer(nb, na) if builtin else crandn(rng, nb, na)
    Y = host(pusch.beamform(dev(X), nb, W=None if builtin else dev(W), n_re=n_re))
    ref = np.swapaxes(O.beamform(W, X[:, :, :n_re]), 1, 2)  # RE-major
    assert_grid(Y, ref)


def test_beamform_long_row_pitch():
    # 16 antennas, rows 2^24 elements apart: offsets past 32 bits take the
    # chunked kernel with 64-bit addressing
    na, nb, nre, ld = 16, 16, 300, 1 << 24
    rng = np.random.default_rng(5)
    Xs = crandn(rng, 1, na, nre)
    X = torch.zeros(1, na, ld, dtype=torch.complex64, device=DEV)
    X[:, :, :nre] = dev(Xs)
    Y = host(pusch.beamform(X, nb, n_re=nre))
    del X
    ref = np.swapaxes(O.beamform(O.dft_beamformer(nb, na), Xs), 1, 2)
    assert_grid(Y, ref)


def test_beamform_full_size_sampled():
    g = torch.Generator(device=DEV)
    g.manual_seed(7)
    batch, na, nre, nb = 16 * 14, 64, 3300, 32
    X = torch.view_as_complex(torch.randn(batch, na, nre, 2, generator=g, device=DEV)).contiguous()
    Y = pusch.beamform(X, nb)
    rng = np.random.default_rng(1)
    bi = rng.integers(0, batch, 40)
    n = rng.integers(0, nre, 40)
    bi[0], n[0], bi[1], n[1] = 0, 0, batch - 1, nre - 1
    Xs = host(X[torch.as_tensor(bi, device=DEV), :, torch.as_tensor(n, device=DEV)])  # [40, na]
    ref = Xs.astype(complex) @ O.dft_beamformer(nb, na).T
    assert_grid(host(Y[torch.as_tensor(bi, device=DEV), torch.as_tensor(n, device=DEV)]), ref)


# ----------------------------------------------------------------------------- LS channel estimate

@pytest.mark.parametrize("nb,nue,nsc,npil,batch", [
    (16, 4, 256, 1, 1),
    (32, 16, 3300, 2, 2),
    (5, 3, 31, 2, 2),  # n_ue not a multiple of n_pilot
    (8, 1, 10, 2, 1),  # one UE: both pilot symbols on every subcarrier (averaged)
    (64, 32, 100, 4, 1),
    (4, 4, 4, 1, 1),  # one pilot subcarrier per UE: pure hold
    (6, 5, 12, 3, 2),
])
def test_chest(nb, nue, nsc, npil, batch):
    rng = np.random.default_rng(nb + 7 * nue + nsc)
    Yp = crandn(rng, batch, npil, nsc, nb)
    amp = rng.uniform(0.5, 2.0, (batch, npil, nsc))
    P = (synth.qam_modulate(rng.integers(0, 2, (batch, npil, nsc, 2)), 2) * amp).astype(np.complex64)
    H = host(pusch.chest(dev(Yp), dev(P), nue))
    for b in range(batch):
        ref = O.ls_channel_estimate(np.swapaxes(Yp[b], 1, 2), P[b], nue)  # [K, NB, NL]
        assert_grid(H[b], np.swapaxes(ref, 1, 2))


# ----------------------------------------------------------------------------- MMSE detection

@pytest.mark.parametrize("nb,nue,nsc,nd,batch,s2", [
    (16, 4, 256, 13, 1, 0.01),
    (32, 16, 3300, 12, 2, 0.01),
    (32, 16, 1001, 12, 1, 0.01),  # 16 UEs, n_sc % 4 != 0: partial last block of the 16-UE kernel
    (16, 16, 1003, 3, 1, 0.1),  # square 16 x 16, n_sc % 4 == 3
    (8, 3, 37, 5, 2, 0.3),
    (64, 32, 50, 12, 1, 0.1),
    (2, 1, 20, 17, 1, 0.5),  # more data symbols than one kernel call takes
    (4, 2, 9, 40, 1, 0.2),
    (6, 6, 7, 3, 1, 1.0),  # square
    (1, 1, 5, 1, 1, 0.0),
])
def test_mmse(nb, nue, nsc, nd, batch, s2):
    rng = np.random.default_rng(nb * 100 + nue)
    H = (crandn(rng, batch, nsc, nue, nb) / np.sqrt(2)).astype(np.complex64)
    Yd = crandn(rng, batch, nd, nsc, nb)
    x, st = pusch.mmse_solve(dev(H), dev(Yd), s2)
    x, st = host(x), host(st)
    for b in range(batch):
        ref, ok = O.mmse_detect(np.swapaxes(H[b], 1, 2), Yd[b], s2)
        assert ok.all() and np.all(st[b] == 0)
        assert_xhat(x[b], ref, TOL_X)


def test_mmse_status_flags():
    rng = np.random.default_rng(3)
    nb, nue, nsc = 8, 4, 40
    H = crandn(rng, 1, nsc, nue, nb)
    H[0, 5, 2, :] = 0  # UE 2 invisible on subcarrier 5, sigma^2 = 0: zero pivot
    H[0, 9, 0, 3] = np.nan
    Yd = crandn(rng, 1, 3, nsc, nb)
    x, st = pusch.mmse_solve(dev(H), dev(Yd), 0.0)
    x, st = host(x), host(st)
    ref, ok = O.mmse_detect(np.swapaxes(H[0], 1, 2), Yd[0], 0.0)
    assert np.array_equal(st[0] == 0, ok)
    assert st[0, 5] == 1 and st[0, 9] == 1 and st[0].sum() == 2
    assert np.all(x[0][:, [5, 9]] == 0)
    keep = np.ones(nsc, bool)
    keep[[5, 9]] = False
    assert_xhat(x[0][:, keep], ref[:, keep], TOL_X)


# ----------------------------------------------------------------------------- fused slot

def run_slot(cfg, data, n_slot=None, W=None):
    xs, ps = data["x_td"], data["pilots"]
    if xs.ndim == 3:
        xs, ps = xs[None], ps[None]
    n_slot = xs.shape[0] if n_slot is None else n_slot
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                      data["sigma2"], n_slot, W=None if W is None else dev(W.astype(np.complex64)))
    xh, st = slot(dev(xs), dev(ps))
    return host(xh), host(st)


def oracle_slot(cfg, s, W=None):
    return O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s["sigma2"], W=W,
                          n_beams=cfg.n_beams)


def check_decisions(got, ref, bits):
    pts, lab = synth.qam_table(bits)
    _, bg = M.hard_decide(got, pts, lab)
    _, br = M.hard_decide(ref, pts, lab)
    err = np.abs(got - ref)
    # a decision may legitimately differ only where the oracle's soft value is
    # within the observed rounding distance of a decision boundary
    near = M.decision_margin(ref, pts) <= 8 * float(err.max()) + 1e-9
    assert np.array_equal(bg[~near], br[~near])
    assert near.mean() < 1e-3
    return bg, br


def test_slot_cfg1_20db():
    cfg = synth.CFG1
    s = synth.make_slot(cfg, 1000)
    xh, st = run_slot(cfg, s)
    ref = oracle_slot(cfg, s)
    assert np.all(st == 0)
    assert_xhat(xh[0], ref["x_hat"], TOL_X)
    bg, br = check_decisions(xh[0], ref["x_hat"], cfg.qam_bits)
    assert np.array_equal(bg, br)
    assert np.array_equal(bg, np.swapaxes(s["bits"], 1, 2))  # error-free at 20 dB


def test_slot_cfg1_noiseless_exact_bits():
    cfg = synth.CFG1.replace(snr_db=None)
    s = synth.make_slot(cfg, 1001)
    xh, st = run_slot(cfg, s)
    x = np.swapaxes(s["data"], 1, 2)
    assert_xhat(xh[0], x, TOL_X)
    pts, lab = synth.qam_table(cfg.qam_bits)
    _, bg = M.hard_decide(xh[0], pts, lab)
    assert np.array_equal(bg, np.swapaxes(s["bits"], 1, 2))


def test_slot_cfg2_two_slots():
    cfg = synth.CFG2
    b = synth.make_batch(cfg, [2000, 2001])
    xh, st = run_slot(cfg, b)
    assert np.all(st == 0)
    for i, seed in enumerate([2000, 2001]):
        s = synth.make_slot(cfg, seed)
        ref = oracle_slot(cfg, s)
        assert_xhat(xh[i], ref["x_hat"], TOL_X)
        check_decisions(xh[i], ref["x_hat"], cfg.qam_bits)


def test_slot_cfg2_full_batch_sampled():
    # the throughput launch: 16 slots in one call; two distinct slots tiled 8x
    cfg = synth.CFG2
    s0, s1 = synth.make_slot(cfg, 2002), synth.make_slot(cfg, 2003)
    xs = np.stack([s0["x_td"], s1["x_td"]] * 8)
    ps = np.stack([s0["pilots"], s1["pilots"]] * 8)
    xh, st = run_slot(cfg, {"x_td": xs, "pilots": ps, "sigma2": s0["sigma2"]})
    assert np.all(st == 0)
    refs = [oracle_slot(cfg, s0)["x_hat"], oracle_slot(cfg, s1)["x_hat"]]
    for i in range(16):
        assert_xhat(xh[i], refs[i % 2], TOL_X, i)
    assert np.array_equal(xh[0], xh[2]) and np.array_equal(xh[1], xh[15])


def test_slot_cfg2_64_slots_sampled():
    # four times the throughput launch (1.9 GB of time-domain input): every
    # slot against the oracle's result for the distinct slot it repeats, and
    # the status of every subcarrier
    cfg = synth.CFG2
    s0, s1 = synth.make_slot(cfg, 2004), synth.make_slot(cfg, 2005)
    xs = np.stack([s0["x_td"], s1["x_td"]] * 32)
    ps = np.stack([s0["pilots"], s1["pilots"]] * 32)
    print("[parity] 64 paper-scale slots in one call", flush=True)
    xh, st = run_slot(cfg, {"x_td": xs, "pilots": ps, "sigma2": s0["sigma2"]})
    del xs
    assert np.all(st == 0)
    refs = [oracle_slot(cfg, s0)["x_hat"], oracle_slot(cfg, s1)["x_hat"]]
    for i in (0, 1, 31, 32, 62, 63):
        assert_xhat(xh[i], refs[i % 2], TOL_X, i)
    assert all(np.array_equal(xh[i], xh[i % 2]) for i in range(64))


@pytest.mark.parametrize("geom", [
    dict(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(0,), qam_bits=2, channel="tdl"),
    dict(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(0, 4, 7, 11), qam_bits=8, channel="tdl"),
    dict(n_ant=8, n_fft=64, n_sc=60, n_beams=8, n_ue=3, pilot_symb=(3, 9), qam_bits=4, channel="flat"),
    # pilot symbols that put a UE's pilot on the same subcarriers: each end of
    # the interpolation averages two (one UE) or four (two UEs) of them
    dict(n_ant=8, n_fft=256, n_sc=100, n_beams=4, n_ue=1, pilot_symb=(2, 11), qam_bits=4, channel="tdl"),
    dict(n_ant=16, n_fft=256, n_sc=200, n_beams=6, n_ue=2, pilot_symb=(0, 4, 7, 11), qam_bits=6, channel="tdl"),
    # odd number of beams: stand-alone estimation kernel and stored estimate
    dict(n_ant=16, n_fft=256, n_sc=256, n_beams=15, n_ue=4, pilot_symb=(2,), qam_bits=4, channel="flat"),
    # more than 64 antennas: chunked beamforming kernel inside the slot
    dict(n_ant=128, n_fft=256, n_sc=200, n_beams=32, n_ue=8, pilot_symb=(2, 11), qam_bits=4, channel="tdl"),
])
def test_slot_other_geometries(geom):
    cfg = synth.CFG1.replace(snr_db=25.0, **geom)
    b = synth.make_batch(cfg, [31, 32, 33])
    xh, st = run_slot(cfg, b)
    assert np.all(st == 0)
    for i, seed in enumerate([31, 32, 33]):
        ref = oracle_slot(cfg, synth.make_slot(cfg, seed))
        assert_xhat(xh[i], ref["x_hat"], TOL_X)


def test_slot_user_beamformer():
    cfg = synth.CFG1.replace(n_beams=12)
    s = synth.make_slot(cfg, 44)
    rng = np.random.default_rng(44)
    q, _ = np.linalg.qr(rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16)))
    W = q[:12].astype(np.complex64)
    xh, st = run_slot(cfg, s, W=W)
    ref = oracle_slot(cfg, s, W=W.astype(complex))
    assert_xhat(xh[0], ref["x_hat"], TOL_X)


def test_slot_equals_chained_stage_calls():
    cfg = synth.CFG2.replace(n_sc=1000)
    s = synth.make_slot(cfg, 5)
    x = dev(s["x_td"][None])
    p = dev(s["pilots"][None])
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                      s["sigma2"], 1)
    xh_slot, st_slot = slot(x, p)
    Xa = pusch.fft(x.reshape(-1, cfg.n_fft), cfg.n_sc).reshape(14, cfg.n_ant, cfg.n_sc)
    Y = pusch.beamform(Xa, cfg.n_beams)  # [14, K, NB]
    Yp = Y[list(cfg.pilot_symb)].unsqueeze(0).contiguous()
    H = pusch.chest(Yp, p, cfg.n_ue)
    Yd = Y[list(cfg.data_symb)].unsqueeze(0).contiguous()
    xh, st = pusch.mmse_solve(H, Yd, s["sigma2"])
    # the slot estimates the channel inside the detection kernel; same arithmetic, so agreement is at the
    # level of FP32 rounding (contraction of the interpolation may differ between the two kernels)
    assert torch.equal(st, st_slot)
    assert M.nrmse(host(xh), host(xh_slot)) <= 1e-6


def test_slot_deterministic_and_profiled():
    cfg = synth.CFG1
    s = synth.make_slot(cfg, 9)
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                      s["sigma2"], 1)
    x, p = dev(s["x_td"][None]), dev(s["pilots"][None])
    pusch.profile_begin(3)
    outs = [slot(x, p)[0].clone() for _ in range(3)]
    calls, ms = pusch.profile_end()
    assert calls == 3 and all(v > 0 for v in ms.values())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2])


def test_slot_empty_batch():
    cfg = synth.CFG1
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, 0.01, 0)
    x = torch.empty(0, 14, 16, 256, dtype=torch.complex64, device=DEV)
    p = torch.empty(0, 1, 256, dtype=torch.complex64, device=DEV)
    xh, st = slot(x, p)
    assert xh.numel() == 0
