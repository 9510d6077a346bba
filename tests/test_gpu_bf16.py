"""GPU checks of pusch_slot_bf16 (bfloat16 active-bin grids between OFDM
demodulation and beamforming, beamforming on BF16 matrix cores with FP32
accumulation, FP32 estimation and detection) against the FP32 chain and the
FP64 oracle.

Tolerance: bfloat16 keeps 8 significant bits, so the grids and W carry a
relative rounding error of at most u = 2^-9 per value, four times FP16's; the
FP16 form's bound (NRMSE 2e-3 of the oracle for u = 2^-11) scales to 8e-3.
The EVM of the detected symbols against the transmitted ones must stay within
0.1 dB of the FP32 chain's at every SNR, as for the FP16 form.
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
TOL_BF16 = 8e-3
EVM_GAP_DB = 0.1


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run(cfg, b, precision, scale=1.0, sigma2=None):
    n = b["x_td"].shape[0]
    s2 = b["sigma2"] if sigma2 is None else sigma2
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, s2, n,
                      precision=precision)
    x = dev(b["x_td"]) * scale if scale != 1.0 else dev(b["x_td"])
    xh, st = slot(x.contiguous(), dev(b["pilots"]))
    return host(xh), host(st)


@pytest.mark.parametrize("snr_db", [10.0, 20.0, 30.0])
def test_bf16_evm_gap_and_oracle(snr_db):
    cfg = synth.CFG2.replace(snr_db=snr_db)
    b = synth.make_batch(cfg, [3500, 3501])
    print(f"[bf16] paper-scale slots at {snr_db} dB", flush=True)
    x32, st32 = run(cfg, b, "fp32")
    xb, stb = run(cfg, b, "bf16")
    assert np.all(st32 == 0) and np.all(stb == 0)
    data = b["data"].transpose(0, 1, 3, 2)  # [slot][D][K][L], the x_hat layout
    gap = M.evm_db(xb, data) - M.evm_db(x32, data)
    print(f"[bf16] EVM FP32 {M.evm_db(x32, data):.3f} dB, gap {gap:.4f} dB", flush=True)
    assert abs(gap) <= EVM_GAP_DB, gap
    for k in range(2):
        ref = O.receive_slot(b["x_td"][k], b["pilots"][k], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                             n_beams=cfg.n_beams)
        assert_xhat(xb[k], ref["x_hat"], TOL_BF16, "bf16")


@pytest.mark.parametrize("log2_scale", [60, -60])
def test_bf16_needs_no_row_scaling(log2_scale):
    # bfloat16 has FP32's exponent range: x_td * 2^s with sigma2 * 2^(2s)
    # gives the same detected symbols up to the rounding of the scaled values
    # (a power of two changes no significand, so the grids round alike)
    cfg = synth.CFG1
    b = synth.make_batch(cfg, [3600])
    base, _ = run(cfg, b, "bf16")
    a = 2.0 ** log2_scale
    got, st = run(cfg, b, "bf16", scale=a, sigma2=b["sigma2"] * a * a)
    assert np.all(st == 0) and np.all(np.isfinite(got))
    assert M.nrmse(got, base) <= 1e-6
    ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                         n_beams=cfg.n_beams)
    assert_xhat(got[0], ref["x_hat"], TOL_BF16)


def test_bf16_small_geometries():
    for geom in (dict(n_ant=8, n_fft=64, n_sc=60, n_beams=8, n_ue=3, pilot_symb=(3, 9)),
                 dict(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(0, 4, 7, 11), qam_bits=8,
                      channel="tdl"),
                 dict(n_beams=15)):
        cfg = synth.CFG1.replace(snr_db=25.0, **geom)
        b = synth.make_batch(cfg, [3700, 3701])
        got, st = run(cfg, b, "bf16")
        assert np.all(st == 0)
        for k in range(2):
            ref = O.receive_slot(b["x_td"][k], b["pilots"][k], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                                 n_beams=cfg.n_beams)
            assert_xhat(got[k], ref["x_hat"], TOL_BF16, geom)


def test_bf16_sits_between_fp16_and_fp32_error():
    # the same slots through the three forms: the bfloat16 grids' error
    # against the oracle exceeds the FP16 grids' (3 fewer significant bits)
    cfg = synth.CFG2.replace(snr_db=30.0)
    b = synth.make_batch(cfg, [3800])
    ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                         n_beams=cfg.n_beams)["x_hat"]
    err = {p: M.nrmse(run(cfg, b, p)[0][0], ref) for p in ("fp32", "mixed", "bf16")}
    print(f"[bf16] NRMSE vs oracle {err}", flush=True)
    assert err["fp32"] < err["mixed"] < err["bf16"] <= TOL_BF16
