"""The precision form's main shape through the whole chain: 64 receive
antennas, 4096-point FFT with 3300 active subcarriers, 32 UEs with 64-QAM on
the 8-tap 300 ns channel, with the square 64 x 64 DFT beamformer and with 32
beams (as many beams as UEs, the ill-conditioned stress point), at 10, 20 and
30 dB, in FP32 and in mixed precision, with and without one step of
iterative refinement.

Every run is scored against the FP64 oracle (NRMSE, largest element error and
worst subcarrier, in units of the reference RMS) and by its EVM against the
transmitted symbols; the table printed per case is the precision form's
per-SNR error statement.
"""
import numpy as np
import pytest
import torch

from checks import assert_xhat
from oracle import metrics as M
from oracle import pusch_oracle as O
from paper_2210_09196_amd import pusch, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL_X = 1e-4
TOL_MIXED = 2e-3


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def run(cfg, b, precision, refine):
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, b["sigma2"],
                      b["x_td"].shape[0], precision=precision, refine=refine)
    xh, st = slot(dev(b["x_td"]), dev(b["pilots"]))
    torch.cuda.synchronize()
    return xh.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("n_beams", [64, 32])
@pytest.mark.parametrize("snr_db", [10.0, 20.0, 30.0])
def test_precision_form_main_shape(n_beams, snr_db):
    cfg = synth.CFG2.replace(n_beams=n_beams, n_ue=32, snr_db=snr_db)
    print(f"[precision] 64 ant / {n_beams} beams / 32 UEs, {snr_db} dB", flush=True)
    b = synth.make_batch(cfg, [3000 + int(snr_db) + n_beams])
    ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                         n_beams=cfg.n_beams)
    cond = np.linalg.cond(O.gram(ref["H"], b["sigma2"]))
    data = np.swapaxes(b["data"][0], 1, 2)  # [D][K][L]
    res = {}
    for precision in ("fp32", "mixed"):
        for refine in (False, True):
            xh, st = run(cfg, b, precision, refine)
            assert np.all(st == 0), (precision, refine)
            e = M.xhat_errors(xh[0], ref["x_hat"])
            e["evm"] = M.evm_db(xh[0], data)
            res[precision, refine] = (xh[0], e)
            print(f"  {precision:5s} refine={int(refine)}: nrmse {e['nrmse']:.2e} max-rel {e['max_rel']:.2e} "
                  f"worst-sc {e['worst_sc']:.2e} EVM {e['evm']:.3f} dB", flush=True)
    print(f"  cond(G) median {np.median(cond):.3g} max {cond.max():.3g}; oracle EVM {M.evm_db(ref['x_hat'], data):.3f} dB",
          flush=True)
    # refinement (automatic beyond a condition estimate of 1e3, or everywhere) brings the FP32 chain
    # within its tolerance at every condition number met here
    assert_xhat(res["fp32", True][0], ref["x_hat"], TOL_X, "fp32 refined")
    assert_xhat(res["fp32", False][0], ref["x_hat"], TOL_X, "fp32 automatic")
    # the mixed chain's EVM stays within 0.1 dB of the FP32 chain's
    assert abs(res["mixed", True][1]["evm"] - res["fp32", True][1]["evm"]) <= 0.1
    assert abs(res["mixed", False][1]["evm"] - res["fp32", False][1]["evm"]) <= 0.1
    if n_beams == 64:  # well conditioned (cond(G) ~ 25)
        assert_xhat(res["mixed", True][0], ref["x_hat"], TOL_MIXED, "mixed refined")
    else:
        # as many beams as UEs: cond(G) reaches 1e4..1e5, and the FP16 rounding of the grids
        # (2^-11 per value) is amplified by it -- refinement removes the solver's error, not
        # the data's, so the mixed chain's distance to the oracle is stated, with a loose bound
        assert res["mixed", True][1]["nrmse"] <= 1e-2


@pytest.mark.parametrize("snr_db", [10.0, 30.0])
def test_precision_form_main_shape_bfloat16(snr_db):
    # the same main shape (64 x 64 DFT beamformer, 32 UEs: the detection's
    # 17..32-UE kernel) through the bfloat16 chain, with and without the
    # matrix-core FFT: EVM within 0.1 dB of FP32, NRMSE within the bfloat16
    # form's bound (8e-3; 1.6e-2 with the FFT's three roundings)
    cfg = synth.CFG2.replace(n_beams=64, n_ue=32, snr_db=snr_db)
    b = synth.make_batch(cfg, [3100 + int(snr_db)])
    ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                         n_beams=cfg.n_beams)
    data = np.swapaxes(b["data"][0], 1, 2)
    x32, st32 = run(cfg, b, "fp32", False)
    assert np.all(st32 == 0)
    e32 = M.evm_db(x32[0], data)
    for fft_mfma, tol in ((False, 8e-3), (True, 1.6e-2)):
        slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                          b["sigma2"], 1, precision="bf16", fft_mfma=fft_mfma)
        xh, st = slot(dev(b["x_td"]), dev(b["pilots"]))
        torch.cuda.synchronize()
        xh, st = xh.cpu().numpy(), st.cpu().numpy()
        assert np.all(st == 0)
        gap = M.evm_db(xh[0], data) - e32
        print(f"[precision] bf16 fft_mfma={int(fft_mfma)} {snr_db} dB: EVM gap {gap:.4f} dB", flush=True)
        assert abs(gap) <= 0.1
        assert_xhat(xh[0], ref["x_hat"], tol, f"bf16 fft_mfma={int(fft_mfma)}")
