"""GPU parity of noise-variance estimation (the NE step of the chain): the
stand-alone pusch_noise_est against the FP64 oracle, and pusch_slot /
pusch_slot_mixed / pusch_cells with the noise variance estimated per slot.

Tolerances.  The estimate is a ratio of two sums of non-negative terms.  Each
|r|^2 term is formed in FP32 from values whose rounding is a few ulp of the
pilot-RE values |y|; with the residual r about 10^(-SNR/20) |y|, the relative
error of a term is about 2 * 2^-23 * 10^(SNR/20), below 1e-5 at the SNRs used
here, and the sums average it down.  Hence 2e-5 relative for the stand-alone
kernel on exact FP32 inputs, and 1e-4 through the FP32 chain (FFT and
beamforming rounding of ~1e-6 of |y| enter every residual).  The
mixed-precision chain rounds the grids to FP16 (2^-11 relative): 2e-3.
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
TOL_NE = 2e-5
TOL_NE_CHAIN = 1e-4
TOL_X = 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def pilot_inputs(rng, batch, n_pilot, n_sc, n_beams, n_ue, sigma2, unit=False):
    """Pilot symbols [batch, n_pilot, n_sc, n_beams] through a channel varying smoothly along k, plus noise."""
    k = np.arange(n_sc)
    Y = np.zeros((batch, n_pilot, n_sc, n_beams), complex)
    if unit:
        p = np.exp(0.5j * np.pi * rng.integers(0, 4, (batch, n_pilot, n_sc)))
    else:
        p = rng.uniform(0.5, 2.0, (batch, n_pilot, n_sc)) * np.exp(2j * np.pi * rng.uniform(size=(batch, n_pilot, n_sc)))
    for b in range(batch):
        a = rng.standard_normal((n_ue, n_beams)) + 1j * rng.standard_normal((n_ue, n_beams))
        c = rng.standard_normal((n_ue, n_beams)) + 1j * rng.standard_normal((n_ue, n_beams))
        for j in range(n_pilot):
            own = (k + j * (n_ue // n_pilot)) % n_ue
            h = a[own] + np.exp(2j * np.pi * k / 97.0)[:, None] * c[own] * 0.3
            Y[b, j] = h * p[b, j][:, None]
    Y += (rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)) * np.sqrt(sigma2 / 2)
    return Y.astype(np.complex64), p.astype(np.complex64)


@pytest.mark.parametrize("batch,n_pilot,n_sc,n_beams,n_ue", [
    (3, 2, 3300, 32, 16),   # paper-scale geometry: staggered comb
    (2, 1, 256, 16, 4),     # small workload: one pilot symbol
    (2, 4, 300, 8, 2),      # four pilot symbols on the same subcarriers: averaged positions
    (2, 2, 301, 15, 3),     # unequal gaps, odd beam count, ragged
    (1, 3, 100, 64, 32),    # widest row, most UEs
    (4, 2, 8, 1, 1),        # one beam, tiny
    (2, 1, 64, 33, 32),     # n_sc == 2 n_ue: every UE has exactly two positions
])
def test_noise_est_matches_oracle(batch, n_pilot, n_sc, n_beams, n_ue):
    rng = np.random.default_rng(n_sc + 7 * n_beams)
    Y, p = pilot_inputs(rng, batch, n_pilot, n_sc, n_beams, n_ue, 0.05)
    got = host(pusch.noise_est(dev(Y), dev(p), n_ue))
    for b in range(batch):
        ref = O.noise_variance_estimate(np.swapaxes(Y[b], 1, 2), p[b], n_ue)
        assert abs(got[b] - ref) <= TOL_NE * ref, (b, got[b], ref)


def test_noise_est_deterministic_and_scaled():
    rng = np.random.default_rng(3)
    Y, p = pilot_inputs(rng, 4, 2, 3300, 32, 16, 0.01, unit=True)
    a = host(pusch.noise_est(dev(Y), dev(p), 16))
    b = host(pusch.noise_est(dev(Y), dev(p), 16))
    assert np.array_equal(a, b)
    # a power-of-two scale of the received values scales the estimate exactly
    c = host(pusch.noise_est(dev(Y * np.float32(4.0)), dev(p), 16))
    assert np.array_equal(c, a * 16)
    assert host(pusch.noise_est(dev(Y[:0]), dev(p[:0]), 16)).shape == (0,)


def run_slot(cfg, b, sigma2, precision="fp32", n_beams=None, time_varying=False):
    nb = cfg.n_beams if n_beams is None else n_beams
    n = b["x_td"].shape[0]
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, nb, cfg.n_ue, cfg.pilot_symb, sigma2, n,
                      precision=precision, time_varying=time_varying, comb_aligned=cfg.comb_aligned)
    xh, st = slot(dev(b["x_td"]), dev(b["pilots"]))
    est = None if slot.sigma2_est is None else host(slot.sigma2_est)
    return host(xh), host(st), est


@pytest.mark.parametrize("geom", [
    dict(),                                               # small workload: flat channel, fused detection
    dict(n_beams=15),                                     # odd beams: stand-alone estimation, raw pilot grids
    dict(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(0, 4, 7, 11), qam_bits=8,
         channel="tdl"),
    dict(n_ant=8, n_fft=256, n_sc=100, n_beams=4, n_ue=1, pilot_symb=(2, 11), qam_bits=4, channel="tdl"),
])
def test_slot_with_estimated_noise_matches_oracle(geom):
    cfg = synth.CFG1.replace(snr_db=20.0, **geom)
    seeds = [61, 62, 63]
    b = synth.make_batch(cfg, seeds)
    xh, st, est = run_slot(cfg, b, None)
    assert np.all(st == 0)
    for i, seed in enumerate(seeds):
        s = synth.make_slot(cfg, seed)
        ref = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, None, n_beams=cfg.n_beams)
        assert abs(est[i] - ref["sigma2"]) <= TOL_NE_CHAIN * ref["sigma2"], (i, est[i], ref["sigma2"])
        assert_xhat(xh[i], ref["x_hat"], TOL_X)


def test_slot_paper_scale_estimated_noise_sampled():
    # the 16-slot launch: two distinct slots tiled 8x; every estimate against the oracle's
    cfg = synth.CFG2
    s0, s1 = synth.make_slot(cfg, 2002), synth.make_slot(cfg, 2003)
    b = {"x_td": np.stack([s0["x_td"], s1["x_td"]] * 8), "pilots": np.stack([s0["pilots"], s1["pilots"]] * 8)}
    xh, st, est = run_slot(cfg, b, None)
    assert np.all(st == 0)
    refs = [O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, None, n_beams=cfg.n_beams)
            for s in (s0, s1)]
    for i in range(16):
        r = refs[i % 2]
        assert abs(est[i] - r["sigma2"]) <= TOL_NE_CHAIN * r["sigma2"], (i, est[i], r["sigma2"])
        assert_xhat(xh[i], r["x_hat"], TOL_X, i)
    assert np.array_equal(est[0::2], np.full(8, est[0])) and np.array_equal(xh[1], xh[15])
    print(f"[ne] paper scale at 20 dB: sigma2 {s0['sigma2']:.4g}, estimates {est[0]:.4g} {est[1]:.4g}", flush=True)


@pytest.mark.parametrize("snr_db", [10.0, 20.0, 30.0])
def test_estimated_noise_evm_against_genie(snr_db):
    # EVM of the detected symbols with the estimated noise variance next to the
    # chain given the true one.  On the selective channel the leave-one-out
    # residual also holds the interpolation error over twice the pilot spacing,
    # so at high SNR the estimate exceeds sigma^2 many times over; that error is
    # effective noise for the detector too, and the EVM must not get worse
    cfg = synth.CFG2.replace(snr_db=snr_db)
    b = synth.make_batch(cfg, [3100, 3101])
    x_g, st_g, _ = run_slot(cfg, b, b["sigma2"])
    x_e, st_e, est = run_slot(cfg, b, None)
    assert np.all(st_g == 0) and np.all(st_e == 0)
    data = b["data"].transpose(0, 1, 3, 2)
    e_g, e_e = M.evm_db(x_g, data), M.evm_db(x_e, data)
    print(f"[ne] {snr_db} dB: sigma2 {b['sigma2']:.4g} est {est.tolist()} EVM genie {e_g:.3f} est {e_e:.3f} dB",
          flush=True)
    assert np.all(est > 0) and np.all(np.isfinite(est))
    assert e_e <= e_g + 0.1


def test_mixed_slot_estimated_noise():
    cfg = synth.CFG2
    b = synth.make_batch(cfg, [3200, 3201])
    x32, _, e32 = run_slot(cfg, b, None)
    x16, st, e16 = run_slot(cfg, b, None, precision="mixed")
    assert np.all(st == 0)
    assert np.all(np.abs(e16 - e32) <= 2e-3 * e32), (e16, e32)
    data = b["data"].transpose(0, 1, 3, 2)
    assert abs(M.evm_db(x16, data) - M.evm_db(x32, data)) <= 0.1


def test_cells_with_estimated_noise_match_single_slot_calls():
    geoms = [
        (dict(), 1, None),
        (dict(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(2, 11), qam_bits=8, channel="tdl"), 2,
         None),
        (dict(n_beams=15), 1, None),
        (dict(n_ant=8, n_fft=64, n_sc=60, n_beams=8, n_ue=3, pilot_symb=(3, 9), qam_bits=4), 1, "genie"),
    ]
    cfgs, batches, cells = [], [], []
    for c, (geom, n_slot, mode) in enumerate(geoms):
        cfg = synth.CFG1.replace(snr_db=20.0, **geom)
        b = synth.make_batch(cfg, [1500 + 10 * c + k for k in range(n_slot)])
        cfgs.append(cfg)
        batches.append(b)
        cells.append(dict(n_ant=cfg.n_ant, n_fft=cfg.n_fft, n_sc=cfg.n_sc, n_symb=cfg.n_symb, n_beams=cfg.n_beams,
                          n_ue=cfg.n_ue, pilot_symb=cfg.pilot_symb, n_slot=n_slot,
                          sigma2=b["sigma2"] if mode == "genie" else None))
    cl = pusch.Cells(cells)
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    xh, st = cl(xs, ps)
    torch.cuda.synchronize()
    for c, (cfg, b, g) in enumerate(zip(cfgs, batches, cells)):
        slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                          g["sigma2"], g["n_slot"])
        alone, alone_st = slot(xs[c], ps[c])
        assert torch.equal(alone, xh[c]) and torch.equal(alone_st, st[c]), c
        if g["sigma2"] is None:
            assert torch.equal(slot.sigma2_est, cl.sigma2_est[c]), c
        else:
            assert cl.sigma2_est[c] is None


# ----------------------------------------------------------------------------- aligned pilot comb

@pytest.mark.parametrize("case", ["estimated", "given", "time_varying", "mixed"])
def test_aligned_comb_slot_matches_oracle(case):
    # the comb without stagger: the channel estimate averages the pilot symbols at each position and
    # the noise estimate compares every pilot RE with the mean at its own subcarrier
    cfg = synth.CFG1.replace(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(2, 11), qam_bits=6,
                             channel="tdl", snr_db=20.0, comb_aligned=True,
                             doppler_hz=200.0 if case == "time_varying" else 0.0)
    seeds = [71, 72]
    b = synth.make_batch(cfg, seeds)
    s2 = b["sigma2"] if case == "given" else None
    xh, st, est = run_slot(cfg, b, s2, precision="mixed" if case == "mixed" else "fp32",
                           time_varying=case == "time_varying")
    assert np.all(st == 0)
    for i, seed in enumerate(seeds):
        s = synth.make_slot(cfg, seed)
        ref = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s2, n_beams=cfg.n_beams,
                             time_varying=case == "time_varying", aligned=True)
        if s2 is None:
            tol = 2e-3 if case == "mixed" else TOL_NE_CHAIN
            assert abs(est[i] - ref["sigma2"]) <= tol * ref["sigma2"], (i, est[i], ref["sigma2"])
        assert_xhat(xh[i], ref["x_hat"], 2e-3 if case == "mixed" else TOL_X, (case, i))


@pytest.mark.parametrize("snr_db", [10.0, 20.0, 30.0])
def test_aligned_comb_noise_estimate_is_accurate_on_the_selective_channel(snr_db):
    # the paper-scale slot on its 8-tap channel (300 ns RMS delay spread): with the aligned comb the
    # estimate holds noise only (within 10 % of sigma^2 at every SNR); the staggered comb's
    # leave-one-out prediction counts the channel's variation over 16 subcarriers as noise
    cfg = synth.CFG2.replace(snr_db=snr_db)
    seeds = [3300, 3301]
    al = cfg.replace(comb_aligned=True)
    b_al = synth.make_batch(al, seeds)
    x_al, st_al, est_al = run_slot(al, b_al, None)
    x_gn, _, _ = run_slot(al, b_al, b_al["sigma2"])
    b_st = synth.make_batch(cfg, seeds)
    x_st, _, est_st = run_slot(cfg, b_st, None)
    s2 = b_al["sigma2"]
    evm = lambda x, b: M.evm_db(x, b["data"].transpose(0, 1, 3, 2))
    print(f"[ne] {snr_db} dB: sigma2 {s2:.4g}; aligned comb est/sigma2 {(est_al / s2).round(4).tolist()} "
          f"EVM {evm(x_al, b_al):.3f} dB (genie {evm(x_gn, b_al):.3f}); staggered est/sigma2 "
          f"{(est_st / s2).round(3).tolist()} EVM {evm(x_st, b_st):.3f} dB", flush=True)
    assert np.all(st_al == 0)
    assert np.all(np.abs(est_al / s2 - 1.0) <= 0.1), est_al / s2
    assert abs(evm(x_al, b_al) - evm(x_gn, b_al)) <= 0.1


def test_cells_with_aligned_comb_match_single_slot_calls():
    geoms = [
        dict(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(2, 11), channel="tdl", comb_aligned=True),
        dict(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(2, 11), channel="tdl"),
        dict(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(2, 7, 11), channel="tdl",
             comb_aligned=True),
    ]
    cfgs, batches, cells = [], [], []
    for c, geom in enumerate(geoms):
        cfg = synth.CFG1.replace(snr_db=20.0, qam_bits=4, **geom)
        b = synth.make_batch(cfg, [1700 + c])
        cfgs.append(cfg)
        batches.append(b)
        cells.append(dict(n_ant=cfg.n_ant, n_fft=cfg.n_fft, n_sc=cfg.n_sc, n_symb=cfg.n_symb, n_beams=cfg.n_beams,
                          n_ue=cfg.n_ue, pilot_symb=cfg.pilot_symb, sigma2=None, n_slot=1,
                          comb_aligned=cfg.comb_aligned))
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    for grouped in (True, False):
        run = pusch.Cells(cells, grouped=grouped)
        xh, st = run(xs, ps)
        for c, (cfg, b) in enumerate(zip(cfgs, batches)):
            alone, alone_st, est = run_slot(cfg, b, None)
            assert np.array_equal(host(xh[c]), alone) and np.array_equal(host(st[c]), alone_st), (grouped, c)
            assert np.array_equal(host(run.sigma2_est[c]), est), (grouped, c)
            ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, None,
                                 n_beams=cfg.n_beams, aligned=cfg.comb_aligned)
            assert abs(est[0] - ref["sigma2"]) <= TOL_NE_CHAIN * ref["sigma2"]
            assert_xhat(alone[0], ref["x_hat"], TOL_X, (grouped, c))
