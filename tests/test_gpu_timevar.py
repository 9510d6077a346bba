"""GPU parity of the chain with a channel estimate per data symbol (the slot
descriptor's time_varying flag) against the FP64 oracle's reading of it:
each pilot symbol gives its own estimate, data symbols interpolate linearly in
time between the pilot symbols around them (held outside), and every data
symbol gets its own Gram matrix and Cholesky factor.  Detected symbols within
NRMSE 1e-4 of the oracle, as the static chain."""
import numpy as np
import pytest
import torch

from oracle import metrics as M
from checks import assert_xhat
from oracle import pusch_oracle as O
from paper_2210_09196_amd import pusch, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL_X = 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run(cfg, b, time_varying, sigma2="given", precision="fp32", fft_mfma=False):
    n = b["x_td"].shape[0]
    s2 = b["sigma2"] if sigma2 == "given" else None
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, s2, n,
                      precision=precision, time_varying=time_varying, fft_mfma=fft_mfma)
    xh, st = slot(dev(b["x_td"]), dev(b["pilots"]))
    return host(xh), host(st)


def oracle(cfg, b, k, sigma2="given"):
    s2 = b["sigma2"] if sigma2 == "given" else None
    return O.receive_slot(b["x_td"][k], b["pilots"][k], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s2,
                          n_beams=cfg.n_beams, time_varying=True)


@pytest.mark.parametrize("geom", [
    # paper-scale geometry with 300 Hz Doppler
    dict(n_ant=64, n_fft=4096, n_sc=3300, n_beams=32, n_ue=16, pilot_symb=(2, 11), qam_bits=6, channel="tdl"),
    # four pilot symbols (three interpolation intervals), 8 UEs
    dict(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(0, 4, 7, 11), qam_bits=4, channel="tdl"),
    # flat channel, pilots late in the slot (first data symbols held)
    dict(n_ant=16, n_fft=256, n_sc=240, n_beams=16, n_ue=4, pilot_symb=(5, 12), qam_bits=4, channel="flat"),
    # 16 symbols: 14 data symbols (more than 12, not a multiple of the four
    # lane groups), 16 UEs, a ragged last block of subcarriers
    dict(n_ant=32, n_fft=1024, n_sc=825, n_beams=32, n_ue=16, n_symb=16, pilot_symb=(1, 14), qam_bits=4,
         channel="tdl"),
    # 11 symbols: 9 data symbols, 6 UEs (padding rows), ragged subcarriers
    dict(n_ant=16, n_fft=1024, n_sc=601, n_beams=8, n_ue=6, n_symb=11, pilot_symb=(2, 8), qam_bits=2,
         channel="tdl"),
])
def test_time_varying_chain_matches_oracle(geom):
    cfg = synth.CFG1.replace(snr_db=25.0, doppler_hz=300.0, **geom)
    b = synth.make_batch(cfg, [41, 42])
    xh, st = run(cfg, b, True)
    assert np.all(st == 0)
    for k in range(2):
        ref = oracle(cfg, b, k)
        assert_xhat(xh[k], ref["x_hat"], TOL_X, k)


def test_time_varying_tracks_doppler_better_than_static():
    cfg = synth.CFG2.replace(doppler_hz=300.0, snr_db=25.0)
    b = synth.make_batch(cfg, [43, 44])
    x_tv, _ = run(cfg, b, True)
    x_st, _ = run(cfg, b, False)
    data = b["data"].transpose(0, 1, 3, 2)
    e_tv, e_st = M.evm_db(x_tv, data), M.evm_db(x_st, data)
    print(f"[timevar] 300 Hz, 25 dB: EVM per-symbol estimate {e_tv:.2f} dB, static {e_st:.2f} dB", flush=True)
    assert e_tv < e_st - 1.0


def test_time_varying_with_one_pilot_symbol_is_the_static_chain():
    cfg = synth.CFG1
    b = synth.make_batch(cfg, [1000])
    x_tv, st = run(cfg, b, True)
    x_st, _ = run(cfg, b, False)
    assert np.all(st == 0)
    assert M.nrmse(x_tv, x_st) <= 1e-6


def test_time_varying_with_estimated_noise_and_mixed_precision():
    cfg = synth.CFG1.replace(n_ant=32, n_fft=1024, n_sc=825, n_beams=16, n_ue=8, pilot_symb=(2, 11), channel="tdl",
                             doppler_hz=200.0, snr_db=20.0)
    b = synth.make_batch(cfg, [45])
    xh, st = run(cfg, b, True, sigma2=None)
    assert np.all(st == 0)
    ref = oracle(cfg, b, 0, sigma2=None)
    assert_xhat(xh[0], ref["x_hat"], TOL_X)
    x16, st16 = run(cfg, b, True, sigma2=None, precision="mixed")
    assert np.all(st16 == 0)
    assert_xhat(x16[0], ref["x_hat"], 2e-3)


@pytest.mark.parametrize("precision,tol", [("mixed", 4e-3), ("bf16", 1.6e-2)])
def test_time_varying_estimated_noise_reduced_precision_and_matrix_core_fft(precision, tol):
    # every option at once on the paper-scale geometry: per-symbol channel,
    # estimated noise, 4-byte grids and the FFT's passes on the matrix cores
    # (tolerances of the matrix-core FFT's tests)
    cfg = synth.CFG2.replace(doppler_hz=300.0, snr_db=25.0)
    b = synth.make_batch(cfg, [46])
    xh, st = run(cfg, b, True, sigma2=None, precision=precision, fft_mfma=True)
    assert np.all(st == 0)
    ref = oracle(cfg, b, 0, sigma2=None)
    assert_xhat(xh[0], ref["x_hat"], tol, precision)


def test_time_varying_status_flags_accumulate_over_symbols():
    # UE 1's estimate from pilot symbol 2 is zero (huge pilots: its LS values
    # round to 0) and sigma^2 = 0: data symbols 0 and 1, which hold that
    # estimate, fail on every subcarrier; later symbols interpolate towards
    # pilot symbol 11 and succeed.  The flags must survive the later symbols
    # (ORed), and only the failing symbols' outputs are zero.
    cfg = synth.CFG1.replace(pilot_symb=(2, 11), snr_db=None)
    b = dict(synth.make_batch(cfg, [46]))
    p = b["pilots"].copy()
    own = np.arange(cfg.n_sc) % cfg.n_ue  # owners on pilot symbol 0 (offset 0)
    p[0, 0, own == 1] = 1e30
    b["pilots"] = p
    b["sigma2"] = 0.0
    xh, st = run(cfg, b, True)
    assert np.all(st == 1)
    assert np.all(xh[0, :2] == 0)
    assert np.all(np.abs(xh[0, 2:]).sum(axis=(1, 2)) > 0)


def test_cells_time_varying_match_single_slot_calls():
    cfg = synth.CFG1.replace(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(2, 11), channel="tdl",
                             doppler_hz=300.0)
    b = synth.make_batch(cfg, [47])
    geo = dict(n_ant=cfg.n_ant, n_fft=cfg.n_fft, n_sc=cfg.n_sc, n_symb=cfg.n_symb, n_beams=cfg.n_beams,
               n_ue=cfg.n_ue, pilot_symb=cfg.pilot_symb, sigma2=b["sigma2"], n_slot=1, time_varying=True)
    x = dev(b["x_td"])
    p = dev(b["pilots"])
    xh, st = pusch.Cells([geo, dict(geo, time_varying=False)])([x, x], [p, p])
    alone, alone_st = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                                 b["sigma2"], 1, time_varying=True)(x, p)
    assert torch.equal(alone, xh[0]) and torch.equal(alone_st, st[0])
    assert not torch.equal(xh[0], xh[1])
